// ppc_batch.hip -- many streams of mixed widths in one persistent launch.
//
// The work of a call is laid out on one axis of "weighted units": stream s
// occupies [cum[s], cum[s+1]) with weight stream_weight + (16-byte body units of
// s); the stream_weight prefix of its range stands for its edge bytes and its
// flush, the rest is its aligned body, unit for unit.  Invalid and empty streams
// weigh nothing.  Block b of a grid of G blocks takes the b-th of G equal shares
// of the axis, so every block reads the same number of bytes give or take one
// stream weight, however uneven the stream lengths are.  A long stream is split
// over many blocks, a block's share covers many short streams.
//
// Two kernels per call:
//   batch_prep  (one block): validates the descriptors, scans their weights into
//               cum[0..m] and, for every block, records the first position its
//               share touches, into first[0..G);  above 4096 streams the same
//               work is split over one block per 2048 positions (prep_chunks,
//               then prep_finish), since a single compute unit is slow to load
//               and weigh tens of thousands of descriptors;
//   batch_main  (G blocks): each block walks the streams of its share; for each
//               it runs the CSA core of the single-stream kernel over its piece of
//               the body (the block's waves take its 64-lane tiles in turn), the
//               block that owns the start of the stream adds its edge bytes, and
//               the block flushes that piece with one atomic per word position.
// Counting uses the 32 dword-bit classes for every width, so streams of any k
// share one code path; the flush folds the classes into the stream's k
// positions with its start rotation.  The carry planes of the circuit go into
// an 8-plane vertical counter per lane (two ops per plane, and few registers, so
// many waves stay resident to hide the latency of short streams); every 255
// carries, and at the end of a piece, the planes are turned into class totals,
// reduced over the wave and added into 64-bit per-wave totals in LDS.
//
// Streams are visited in the order pos -> (pos * P) mod m for a fixed prime P
// larger than any m, so a block's share never holds a long run of neighbouring
// descriptors: a list sorted by length spreads its short streams over all blocks
// as a shuffled one does.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ppc_device.h"
#include "ppc_internal.h"

struct ppc_plan {
    int device = -1;
    uint32_t max_streams = 0;
    uint32_t flags = 0;
    int cus = 0;
    int gmax = 0;
    void* scratch = nullptr;
    uint64_t* cum = nullptr;                  // [max_streams + 1]
    uint32_t* first = nullptr;                // [gmax]
    uint32_t* rejected = nullptr;             // [1]
    uint64_t* part = nullptr;                 // [chunks]: weight of each prep chunk
    uint32_t* part_bad = nullptr;             // [chunks]: rejected descriptors per chunk
    unsigned long long* sink = nullptr;       // [gmax][32], autotune target, one row per block
    ppc_batch_config cfg{};
    int cfg_version = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    const ppc_desc* g_descs = nullptr;
    uint32_t g_m = 0;
    int g_version = -1;
    char arch[64] = {0};
};

namespace ppc {

constexpr int kBatchMaxThreads = 256;
constexpr int kBatchClasses = 32;  // dword-bit classes of the batched kernel
constexpr int kPrepThreads = 1024;
constexpr uint32_t kMaxPlanStreams = 1u << 26;
constexpr int kMaxBlocksPerCu = 16;

struct DevStream {
    Edges edges;
    const u32x4* body;
    uint64_t units;
    uint32_t rot;
};

// The same head / body / tail split as the host's split_stream.
__device__ __forceinline__ DevStream split_dev(const void* ptr, uint64_t nbytes, int k) {
    DevStream s;
    const uintptr_t p = (uintptr_t)ptr, end = p + nbytes;
    const uintptr_t a0 = (p + 15) & ~(uintptr_t)15;
    s.rot = 8u * (uint32_t)(p % (uintptr_t)(k / 8));
    s.edges.head = (const uint8_t*)ptr;
    if (a0 >= end) {
        s.edges.head_len = (uint32_t)nbytes;
        s.edges.tail = (const uint8_t*)end;
        s.edges.tail_len = 0;
        s.body = (const u32x4*)a0;
        s.units = 0;
        return s;
    }
    const uintptr_t a1 = end & ~(uintptr_t)15;
    s.edges.head_len = (uint32_t)(a0 - p);
    s.edges.tail = (const uint8_t*)a1;
    s.edges.tail_len = (uint32_t)(end - a1);
    s.body = (const u32x4*)a0;
    s.units = (uint64_t)(a1 - a0) / 16;
    return s;
}

// Descriptor checks (the device-side counterpart of check_stream_args).
__device__ __forceinline__ bool desc_valid(const ppc_desc& d, uint64_t* nbytes) {
    *nbytes = 0;
    if (d.reserved != 0) return false;
    if (d.k != 8 && d.k != 16 && d.k != 32) return false;
    if (d.n == 0) return true;
    const uint64_t wb = d.k / 8;
    if (d.n > ~0ull / wb) return false;
    const uint64_t nb = d.n * wb;
    const uintptr_t p = (uintptr_t)d.ptr, c0 = (uintptr_t)d.counts;
    if (!p || !c0 || (c0 & 7u)) return false;
    if (p + nb < p) return false;
    const uintptr_t c1 = c0 + 8u * d.k;
    if (c0 < p + nb && p < c1) return false;
    *nbytes = nb;
    return true;
}

__device__ __forceinline__ uint64_t share_lo(uint64_t b, uint64_t total, uint64_t G) {
    const uint64_t base = total / G, extra = total % G;
    return b * base + (b < extra ? b : extra);
}

// Exclusive scan of one value per thread over the block; *total receives the sum.
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* total, uint64_t* sh) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) sh[wave] = x;
    __syncthreads();
    if (wave == 0) {
        uint64_t w = lane < nwaves ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_up(w, o, kWave);
            if (lane >= o) w += y;
        }
        if (lane < nwaves) sh[lane] = w;
    }
    __syncthreads();
    const uint64_t before = wave ? sh[wave - 1] : 0;
    *total = sh[nwaves - 1];
    __syncthreads();
    return before + x - v;
}

// Visiting order of the streams: position pos holds stream (pos * kVisitPrime) mod m,
// a permutation of [0, m) because the prime exceeds every m a plan accepts.
constexpr uint64_t kVisitPrime = 2654435761ull;

__device__ __forceinline__ uint32_t stream_at(uint32_t pos, uint32_t m) {
    return (uint32_t)(((uint64_t)pos * kVisitPrime) % m);
}

// Weight of one descriptor on the axis (0 for empty or invalid ones).
__device__ __forceinline__ uint64_t weight_of(const ppc_desc& d, uint64_t weight, uint32_t* bad) {
    uint64_t nb;
    if (!desc_valid(d, &nb)) {
        ++*bad;
        return 0;
    }
    return nb ? weight + split_dev(d.ptr, nb, (int)d.k).units : 0;
}

constexpr int kPrepPerThread = 4;
constexpr uint32_t kPrepLdsPositions = kPrepThreads * kPrepPerThread;  // cum kept in LDS up to here

// Two passes in one block.  Pass 1 writes the weight of every position into cum
// (four descriptor loads in flight per thread).  Pass 2 turns cum into its
// exclusive prefix sums, four consecutive positions per thread; up to 4096
// positions the prefix array is also kept in LDS.  Then every block's first
// position -- the last one starting at or before the block's share -- is found
// by binary search (in LDS when it holds the array).  With zero_counts, the
// counters of every valid descriptor are cleared first (for callers whose
// descriptors own distinct counters and want fresh counts, like the serving
// loop; the public entry point adds into counters and never sets it).
__global__ void __launch_bounds__(kPrepThreads)
batch_prep(const ppc_desc* __restrict__ descs, uint32_t m, uint64_t weight, uint64_t* cum,
           uint32_t* first, uint32_t G, uint32_t* rejected, int zero_counts) {
    constexpr int R = kPrepPerThread;
    __shared__ uint64_t sh[kPrepThreads / kWave];
    __shared__ uint64_t lcum[kPrepLdsPositions + 1];
    __shared__ uint32_t bad_total;
    if (threadIdx.x == 0) bad_total = 0;
    const uint32_t T = blockDim.x;
    const bool in_lds = m <= kPrepLdsPositions;
    uint64_t local = 0;
    uint32_t bad = 0;
    for (uint32_t c0 = 0; c0 < m; c0 += T * R) {
        ppc_desc d[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = c0 + r * T + threadIdx.x;
            if (i < m) d[r] = descs[stream_at(i, m)];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = c0 + r * T + threadIdx.x;
            if (i < m) {
                const uint64_t w = weight_of(d[r], weight, &bad);
                cum[i] = w;
                local += w;
                if (zero_counts && w)  // valid and non-empty: counts checked by desc_valid
                    for (uint32_t p = 0; p < d[r].k; ++p) d[r].counts[p] = 0;
            }
        }
    }
    uint64_t total;
    (void)block_exclusive_scan(local, &total, sh);  // barriers: pass-1 writes are visible
    uint64_t carry = 0;
    for (uint32_t c0 = 0; c0 < m; c0 += T * R) {
        const uint32_t p0 = c0 + threadIdx.x * R;
        uint64_t w[R], sum = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w[r] = p0 + r < m ? cum[p0 + r] : 0;
            sum += w[r];
        }
        uint64_t round_total;
        uint64_t run = carry + block_exclusive_scan(sum, &round_total, sh);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (p0 + r < m) {
                cum[p0 + r] = run;
                if (in_lds) lcum[p0 + r] = run;
                run += w[r];
            }
        }
        carry += round_total;
    }
    if (threadIdx.x == 0) {
        cum[m] = total;
        if (in_lds) lcum[m] = total;
    }
    if (bad) atomicAdd(&bad_total, bad);
    __syncthreads();
    if (threadIdx.x == 0) rejected[0] = bad_total;
    const uint64_t base = total / G, extra = total % G;
    for (uint32_t b = threadIdx.x; b < G; b += T) {
        const uint64_t lo = (uint64_t)b * base + (b < extra ? b : extra);
        uint32_t l = 0, h = m;  // last position l < m with cum[l] <= lo
        while (h - l > 1) {
            const uint32_t mid = l + (h - l) / 2;
            const uint64_t c = in_lds ? lcum[mid] : cum[mid];
            if (c <= lo) l = mid; else h = mid;
        }
        first[b] = l;
    }
}

// ---- batch preparation over several blocks (more than kPrepLdsPositions streams)

constexpr uint32_t kChunk = 2 * kPrepThreads;  // positions per block

// Smallest block b in [0, G] whose share starts at or after axis position c
// (c <= total); block b's share starts at b * base + min(b, extra).
__device__ __forceinline__ uint32_t share_at_or_after(uint64_t c, uint64_t total, uint64_t G) {
    const uint64_t base = total / G, extra = total % G;
    if (base == 0) return (uint32_t)c;
    const uint64_t wide = extra * (base + 1);  // blocks 0 .. extra-1 take base + 1
    if (c <= wide) return (uint32_t)((c + base) / (base + 1));
    return (uint32_t)(extra + (c - wide + base - 1) / base);
}

// Pass 1: the weight of every position of this block's chunk into cum, the chunk's
// total into part[chunk], its rejected descriptors into part_bad[chunk].  Both
// descriptor loads of a thread are in flight together.
__global__ void __launch_bounds__(kPrepThreads)
prep_chunks(const ppc_desc* __restrict__ descs, uint32_t m, uint64_t weight, uint64_t* cum,
            uint64_t* part, uint32_t* part_bad, int zero_counts) {
    __shared__ uint64_t sh[kPrepThreads / kWave];
    __shared__ uint32_t bad_total;
    if (threadIdx.x == 0) bad_total = 0;
    const uint32_t base = blockIdx.x * kChunk;
    ppc_desc d[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t i = base + r * kPrepThreads + threadIdx.x;
        if (i < m) d[r] = descs[stream_at(i, m)];
    }
    uint64_t local = 0;
    uint32_t bad = 0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t i = base + r * kPrepThreads + threadIdx.x;
        if (i < m) {
            const uint64_t w = weight_of(d[r], weight, &bad);
            cum[i] = w;
            local += w;
            if (zero_counts && w)
                for (uint32_t p = 0; p < d[r].k; ++p) d[r].counts[p] = 0;
        }
    }
    uint64_t total;
    (void)block_exclusive_scan(local, &total, sh);  // its barriers order bad_total too
    if (bad) atomicAdd(&bad_total, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x] = total;
        part_bad[blockIdx.x] = bad_total;
    }
}

// Pass 2, one block per chunk: the chunk's offset on the axis (the weights of the
// chunks before it), the exclusive prefix sums of its positions into cum (and into
// LDS), and first[b] for every block b whose share starts inside the chunk's range
// of the axis, by binary search in LDS.  The last chunk writes cum[m], the rejected
// count, and first[b] = m - 1 for the shares that start at the end of the axis
// (when the axis is shorter than the grid).
__global__ void __launch_bounds__(kPrepThreads)
prep_finish(uint32_t m, uint64_t* cum, const uint64_t* __restrict__ part,
            const uint32_t* __restrict__ part_bad, uint32_t chunks, uint32_t* first, uint32_t G,
            uint32_t* rejected) {
    __shared__ uint64_t sh[kPrepThreads / kWave];
    __shared__ uint64_t lcum[kChunk];
    const uint32_t c = blockIdx.x, T = blockDim.x;
    uint64_t before = 0, all = 0;
    uint32_t bad = 0;
    for (uint32_t j = threadIdx.x; j < chunks; j += T) {
        all += part[j];
        if (j < c) before += part[j];
        bad += part_bad[j];
    }
    uint64_t off, total;
    (void)block_exclusive_scan(before, &off, sh);
    (void)block_exclusive_scan(all, &total, sh);
    const uint32_t base = c * kChunk;
    const uint32_t n = min(kChunk, m - base);
    const uint32_t p = 2 * threadIdx.x;
    const uint64_t w0 = p < n ? cum[base + p] : 0, w1 = p + 1 < n ? cum[base + p + 1] : 0;
    uint64_t chunk_total;
    const uint64_t c0 = off + block_exclusive_scan(w0 + w1, &chunk_total, sh);
    if (p < n) {
        cum[base + p] = c0;
        lcum[p] = c0;
    }
    if (p + 1 < n) {
        cum[base + p + 1] = c0 + w0;
        lcum[p + 1] = c0 + w0;
    }
    if (c == chunks - 1) {
        if (threadIdx.x == 0) cum[m] = total;
        uint64_t nb;
        (void)block_exclusive_scan(bad, &nb, sh);
        if (threadIdx.x == 0) rejected[0] = (uint32_t)nb;
        for (uint32_t b = share_at_or_after(total, total, G) + threadIdx.x; b < G; b += T)
            first[b] = m - 1;
    }
    __syncthreads();
    if (chunk_total == 0) return;
    const uint32_t b1 = min(share_at_or_after(off + chunk_total, total, G), G);
    for (uint32_t b = share_at_or_after(off, total, G) + threadIdx.x; b < b1; b += T) {
        const uint64_t lo = share_lo(b, total, G);
        uint32_t l = 0, h = n;  // last position l < n of the chunk with lcum[l] <= lo
        while (h - l > 1) {
            const uint32_t mid = l + (h - l) / 2;
            if (lcum[mid] <= lo) l = mid; else h = mid;
        }
        first[b] = base + l;
    }
}

// descs, cum and first are read-only for the whole launch and never alias the
// counters, which lets the per-stream bookkeeping use scalar loads.  sink, when
// not NULL, receives every flush instead of the descriptors' counters, in one
// row of 32 per block (so that timing runs see the same atomic traffic as real
// ones, spread over many addresses).
// The block's share [lo, hi) of the axis: every stream it touches, from position
// pos on, counted into the stream's counters (or into sink).  cum: the prefix
// array, in global memory or in LDS; desc_at(pos): the descriptor at a position.
// With COPY, dst_at(pos) gives the destination of the stream's bytes (the same
// address as the source modulo 16): every byte the block reads of the stream is
// also stored there, so a copy and its count cost one read of the source.
template <int LOGD, bool COPY, typename Cum, typename DescAt, typename DstAt>
__device__ __forceinline__ void walk_share(DescAt desc_at, DstAt dst_at, Cum cum,
                                           uint32_t pos, uint32_t m, uint64_t lo, uint64_t hi,
                                           uint64_t weight, unsigned long long* sink,
                                           uint64_t b,
                                           unsigned long long (*acc)[kBatchClasses]) {
    constexpr int C = kBatchClasses;
    constexpr int L = 8;
    // A vertical counter of L planes holds 2^L - 1 carries: chunks of at most
    // 2^L - 2 tiles leave room for the one masked tail tile.
    constexpr uint64_t kChunk = (1u << L) - 2;
    constexpr int G2 = kWave / C;               // lanes per class after the reduce
    constexpr int U = (1 << LOGD) / 4;
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    uint64_t w0 = cum[pos], w1 = cum[pos + 1];
    for (; pos < m && w0 < hi; ++pos) {
        // the next position's bookkeeping is requested before this one is worked on
        const uint64_t w2 = pos + 2 <= m ? cum[pos + 2] : w1;
        if (w1 > lo && w1 > w0) {
            const ppc_desc d = desc_at(pos);
            const int k = (int)d.k;
            const DevStream st = split_dev(d.ptr, d.n * (uint64_t)(k / 8), k);
            intptr_t delta = 0;  // destination - source, a multiple of 16
            if constexpr (COPY) delta = (intptr_t)dst_at(pos) - (intptr_t)d.ptr;
            const uint64_t bw0 = w0 + weight;  // first body unit of the stream on the axis
            const uint64_t ub = lo > bw0 ? lo - bw0 : 0;
            const uint64_t ue = hi >= w1 ? st.units : (hi > bw0 ? hi - bw0 : 0);
            const bool own_edges = lo <= w0;  // this share holds the stream's start
            if (own_edges || ue > ub) {
                if (lane % G2 == 0) acc[wave][lane / G2] = 0;
                uint32_t B[LOGD], V[L];
#pragma unroll
                for (int j = 0; j < LOGD; ++j) B[j] = 0;
#pragma unroll
                for (int j = 0; j < L; ++j) V[j] = 0;
                auto count_tile = [&](const u32x4(&v)[U]) {
                    uint32_t dw[4 * U];
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        dw[4 * j + 0] = v[j].x;
                        dw[4 * j + 1] = v[j].y;
                        dw[4 * j + 2] = v[j].z;
                        dw[4 * j + 3] = v[j].w;
                    }
                    vertical_add<L>(V, Circuit<LOGD>::run(B, dw));
                };
                auto consume = [&](const u32x4(&v)[U], const u32x4* at) {
                    if constexpr (COPY) store_tile<U>(v, at, delta);
                    count_tile(v);
                };
                if (ue > ub) {
                    const u32x4* base = st.body + ub;
                    const uint64_t len = ue - ub, full = len / TILE, rem = len - full * TILE;
                    // this wave's tiles, in chunks of at most kChunk carries, the vertical
                    // counter drained into the per-wave totals after each chunk
                    uint64_t mine = (uint64_t)wave < full ? (full - wave + wpb - 1) / wpb : 0;
                    const u32x4* p = base + (uint64_t)wave * TILE + lane;
                    const uint64_t stride = (uint64_t)wpb * TILE;
                    while (mine > 0) {
                        const uint64_t n = mine < kChunk ? mine : kChunk;
                        walk_n<U>(p, n, stride, consume);
                        p += n * stride;
                        mine -= n;
                        if (mine > 0) {
                            uint32_t t[C] = {};
                            add_plane_totals<C, L>(t, V, LOGD);
                            const uint32_t v = wave_reduce_scatter<C>(t, lane);
                            if (lane % G2 == 0) acc[wave][lane / G2] += v;
#pragma unroll
                            for (int j = 0; j < L; ++j) V[j] = 0;
                        }
                    }
                    if (rem != 0 && (uint64_t)wave == full % (uint64_t)wpb) {
                        u32x4 t[U];
                        const u32x4* at = base + full * TILE + lane;
                        load_tile_masked<U>(t, at, lane, rem);
                        if constexpr (COPY) store_tile_masked<U>(t, at, delta, lane, rem);
                        count_tile(t);
                    }
                }
                // running planes (weights 2^j), vertical counter (2^(LOGD + j)), edges (1)
                uint32_t e = 0u;
                if (own_edges && wave == 0)
                    e = COPY ? edge_dword_copy(st.edges, lane, delta) : edge_dword(st.edges, lane);
                uint32_t t[C];
#pragma unroll
                for (int i = 0; i < C; ++i) t[i] = __builtin_popcount(e & mask_of<C>(i));
                add_plane_totals<C, L>(t, V, LOGD);
                add_plane_totals<C, LOGD>(t, B, 0);
                const uint32_t v = wave_reduce_scatter<C>(t, lane);
                if (lane % G2 == 0) acc[wave][lane / G2] += v;
                __syncthreads();
                block_flush64<C>(acc, wpb, k, st.rot,
                                 sink ? sink + b * C : (unsigned long long*)d.counts);
                __syncthreads();
            }
        }
        w0 = w1;
        w1 = w2;
    }
}

// dsts (COPY only): per stream index, where the stream's bytes are copied to.
template <int LOGD, bool COPY>
__global__ void __launch_bounds__(kBatchMaxThreads)
batch_main(const ppc_desc* __restrict__ descs, uint8_t* const* __restrict__ dsts,
           const uint64_t* __restrict__ cum, const uint32_t* __restrict__ first, uint64_t weight,
           unsigned long long* sink, uint32_t m) {
    const uint64_t G = gridDim.x, b = blockIdx.x;
    const uint64_t total = cum[m];
    const uint64_t lo = share_lo(b, total, G), hi = share_lo(b + 1, total, G);
    if (lo >= hi) return;  // whole block: no barrier is reached
    __shared__ unsigned long long acc[kBatchMaxThreads / kWave][kBatchClasses];
    walk_share<LOGD, COPY>([&](uint32_t pos) { return descs[stream_at(pos, m)]; },
                           [&](uint32_t pos) { return dsts[stream_at(pos, m)]; }, cum, first[b],
                           m, lo, hi, weight, sink, b, acc);
}

// Circuit depths 4, 8, 16 and 32 dwords per lane (LOGD 2 .. 5).
static int logd_of(int depth) { return logd_of_depth(depth); }

static const void* main_kernel(int depth, bool copy) {
    static const void* const plain[4] = {(const void*)batch_main<2, false>,
                                         (const void*)batch_main<3, false>,
                                         (const void*)batch_main<4, false>,
                                         (const void*)batch_main<5, false>};
    static const void* const copying[4] = {(const void*)batch_main<2, true>,
                                           (const void*)batch_main<3, true>,
                                           (const void*)batch_main<4, true>,
                                           (const void*)batch_main<5, true>};
    return (copy ? copying : plain)[logd_of(depth) - 2];
}

// Small batches in one kernel, for callers whose counters are already zero: every
// block reads all m <= kSmallBatch descriptors into LDS and weighs them (the
// preparation of batch_prep, redone per block from the same descriptors, so all
// blocks agree), keeps the prefix array in LDS, finds its own first position and
// walks its share as batch_main does.  No preparation kernel, and no gap between
// two kernels.  The descriptors are read once per block, so they may live in
// pinned host memory (the serving executor's staging buffer).

template <int LOGD, bool COPY>
__global__ void __launch_bounds__(kBatchMaxThreads)
batch_small(const ppc_desc* __restrict__ descs, uint8_t* const* __restrict__ dsts, uint32_t m,
            uint64_t weight) {
    __shared__ uint64_t lcum[kSmallBatch + 1];
    __shared__ ppc_desc ldesc[kSmallBatch];  // position order
    __shared__ uint8_t* ldst[COPY ? kSmallBatch : 1];
    __shared__ uint64_t sh[kBatchMaxThreads / kWave];
    __shared__ unsigned long long acc[kBatchMaxThreads / kWave][kBatchClasses];
    const uint32_t T = blockDim.x, t = threadIdx.x;
    const uint32_t R = (m + T - 1) / T;  // consecutive positions per thread
    uint64_t local = 0;
    uint32_t bad = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t p = t * R + r;
        if (p < m) {
            const uint32_t i = stream_at(p, m);
            const ppc_desc d = descs[i];
            ldesc[p] = d;
            if constexpr (COPY) ldst[p] = dsts[i];
            const uint64_t w = weight_of(d, weight, &bad);
            lcum[p] = w;
            local += w;
        }
    }
    uint64_t total;
    uint64_t run = block_exclusive_scan(local, &total, sh);  // barriers order the writes
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t p = t * R + r;
        if (p < m) {
            const uint64_t w = lcum[p];
            lcum[p] = run;
            run += w;
        }
    }
    if (t == 0) lcum[m] = total;
    __syncthreads();
    const uint64_t G = gridDim.x, b = blockIdx.x;
    const uint64_t lo = share_lo(b, total, G), hi = share_lo(b + 1, total, G);
    if (lo >= hi) return;  // whole block: no barrier is reached
    uint32_t l = 0, h = m;  // last position l < m with lcum[l] <= lo
    while (h - l > 1) {
        const uint32_t mid = l + (h - l) / 2;
        if (lcum[mid] <= lo) l = mid; else h = mid;
    }
    walk_share<LOGD, COPY>([&](uint32_t pos) { return ldesc[pos]; },
                           [&](uint32_t pos) { return ldst[COPY ? pos : 0]; },
                           (const uint64_t*)lcum, l, m, lo, hi, weight, nullptr, b, acc);
}

static const void* small_kernel(int depth, bool copy) {
    static const void* const plain[4] = {(const void*)batch_small<2, false>,
                                         (const void*)batch_small<3, false>,
                                         (const void*)batch_small<4, false>,
                                         (const void*)batch_small<5, false>};
    static const void* const copying[4] = {(const void*)batch_small<2, true>,
                                           (const void*)batch_small<3, true>,
                                           (const void*)batch_small<4, true>,
                                           (const void*)batch_small<5, true>};
    return (copy ? copying : plain)[logd_of(depth) - 2];
}

static int check_config(const ppc_batch_config& c) {
    if (logd_of(c.depth) < 0) return PPC_ERR_ARG;
    if (c.block_threads != 64 && c.block_threads != 128 && c.block_threads != 256)
        return PPC_ERR_ARG;
    if (c.blocks_per_cu < 1 || c.blocks_per_cu > kMaxBlocksPerCu) return PPC_ERR_ARG;
    if (c.stream_weight < 1 || c.stream_weight > 65536) return PPC_ERR_ARG;
    return PPC_OK;
}

// Device scratch of one batched call: the prefix array cum[m+1], the per-block
// start table first[G], the rejected count, and the chunk weights and rejected
// counts of the split preparation (above kPrepLdsPositions streams).
struct BatchScratch {
    uint64_t* cum;
    uint32_t* first;
    uint32_t* rejected;
    uint64_t* part;
    uint32_t* part_bad;
};

// Enqueues the preparation and the persistent kernel of one batched call on s,
// with the grid of c (cut to max_blocks when that is not 0).
// dsts, when not NULL, gives per stream index where its bytes are copied to.
static int enqueue_with(const BatchScratch& sc, const ppc_batch_config& c, int cus,
                        const ppc_desc* descs, uint32_t m, hipStream_t s,
                        unsigned long long* sink, int zero_counts, uint32_t max_blocks,
                        uint8_t* const* dsts = nullptr) {
    uint32_t G = (uint32_t)(c.blocks_per_cu * cus);
    if (max_blocks && max_blocks < G) G = max_blocks;
    uint64_t weight = (uint64_t)c.stream_weight;
    uint64_t* cum_w = sc.cum;
    uint32_t* first_w = sc.first;
    uint32_t* rej = sc.rejected;
    if (m <= kPrepLdsPositions) {
        void* pargs[] = {(void*)&descs, &m, &weight, &cum_w, &first_w, &G, &rej, &zero_counts};
        PPC_HIP(hipLaunchKernel((const void*)batch_prep, dim3(1), dim3(kPrepThreads), pargs, 0, s));
    } else {
        uint32_t chunks = (m + kChunk - 1) / kChunk;
        uint64_t* part_w = sc.part;
        uint32_t* bad_w = sc.part_bad;
        void* a1[] = {(void*)&descs, &m, &weight, &cum_w, &part_w, &bad_w, &zero_counts};
        PPC_HIP(hipLaunchKernel((const void*)prep_chunks, dim3(chunks), dim3(kPrepThreads), a1, 0, s));
        const uint64_t* part = sc.part;
        const uint32_t* part_bad = sc.part_bad;
        void* a2[] = {&m, &cum_w, (void*)&part, (void*)&part_bad, &chunks, &first_w, &G, &rej};
        PPC_HIP(hipLaunchKernel((const void*)prep_finish, dim3(chunks), dim3(kPrepThreads), a2, 0,
                                s));
    }
    const uint64_t* cum = sc.cum;
    const uint32_t* first = sc.first;
    void* margs[] = {(void*)&descs, (void*)&dsts, (void*)&cum, (void*)&first, &weight, &sink, &m};
    PPC_HIP(hipLaunchKernel(main_kernel(c.depth, dsts != nullptr), dim3(G), dim3(c.block_threads),
                            margs, 0, s));
    return PPC_OK;
}

static int enqueue(ppc_plan* pl, const ppc_desc* descs, uint32_t m, hipStream_t s,
                   unsigned long long* sink, int zero_counts = 0, uint32_t max_blocks = 0,
                   uint8_t* const* dsts = nullptr) {
    const BatchScratch sc{pl->cum, pl->first, pl->rejected, pl->part, pl->part_bad};
    return enqueue_with(sc, pl->cfg, pl->cus, descs, m, s, sink, zero_counts, max_blocks, dsts);
}

// ---- the batched count without a plan: scratch in a file-scope device array
//
// Layout of `scratch` (each part 256-byte aligned): cum[PPC_STATIC_MAX_STREAMS + 1],
// first[kStaticMaxBlocks], the rejected count, and the split preparation's chunk
// weights and rejected counts.  The preparation kernels write every entry a call
// reads before the persistent kernel reads it, so nothing needs clearing between
// calls.
constexpr uint32_t kStaticMaxBlocks = 4096;  // 16 blocks per CU on 256 CUs
constexpr uint32_t kStaticChunks = (PPC_STATIC_MAX_STREAMS + kChunk - 1) / kChunk;
constexpr size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kStaticCumOff = 0;
constexpr size_t kStaticFirstOff = round256(((size_t)PPC_STATIC_MAX_STREAMS + 1) * 8);
constexpr size_t kStaticRejOff = kStaticFirstOff + round256((size_t)kStaticMaxBlocks * 4);
constexpr size_t kStaticPartOff = kStaticRejOff + 256;
constexpr size_t kStaticPartBadOff = kStaticPartOff + round256((size_t)kStaticChunks * 8);
constexpr size_t kStaticBytes = kStaticPartBadOff + round256((size_t)kStaticChunks * 4);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// The device address of `scratch` on device dev (each device holds its own copy),
// looked up once per device with that device current.  On the host the array's
// name is not a device address; only this pointer is passed to kernels.
static int static_scratch(int dev, char** out) {
    static std::mutex mu;
    static char* addr[64] = {};
    if (dev < 0 || dev >= 64) return PPC_ERR_ARG;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        PPC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return PPC_ERR_HIP;
        addr[dev] = (char*)p;
    }
    *out = addr[dev];
    return PPC_OK;
}

// The autotuner's choice on MI355X for a 20,000-stream uneven mix, in every run
// (ppc_plan_autotune picks per workload): 16 dwords per lane per step, one-wave
// blocks, 4 per CU, and a stream costed like 32 KiB of body -- about what a block
// streams while a stream's bookkeeping, first loads and flush take.  Against a
// stream costed like 64 KiB the same mix ran 1.5-2% faster (6983-7018 against
// 6852-6886 GB/s, libraries compared in one process on four machines).
static ppc_batch_config default_config() { return ppc_batch_config{16, 64, 4, 2048}; }

static int device_of(ppc_plan* pl) {
    int dev = -1;
    PPC_HIP(hipGetDevice(&dev));
    if (dev != pl->device) return PPC_ERR_STATE;
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

namespace ppc {
// The batched count with every valid descriptor's counters cleared first, for
// callers whose descriptors own distinct counters (the serving executor); never
// captured into a graph.  With the batch's input bytes known (bytes > 0), the grid
// is cut to about kFreshUnitsPerWave weighted units per wave: a small batch
// spread over the whole grid would split each stream over hundreds of blocks,
// whose flushes then queue on the same few counters.  One 4 KiB tile per wave
// (at depth 16) measured best in the serving loop at 50,000 requests/s: median
// latency 1-3% below four tiles per wave and 7% below eight, level with two, with
// the tail and the saturated rate unchanged; half a tile was no better.
constexpr uint64_t kFreshUnitsPerWave = 256;  // 4 KiB of body per wave

int batch_fresh(ppc_plan* pl, const ppc_desc* d_descs, uint32_t m, hipStream_t s,
                uint64_t bytes, uint8_t* const* dsts) {
    if (!pl || !d_descs) return PPC_ERR_NULL;
    if (m == 0) return PPC_OK;
    if (m > pl->max_streams) return PPC_ERR_ARG;
    uint32_t max_blocks = 0;
    if (bytes) {
        const uint64_t units = (uint64_t)m * (uint64_t)pl->cfg.stream_weight + bytes / 16;
        const uint64_t per_block = kFreshUnitsPerWave * (uint64_t)(pl->cfg.block_threads / kWave);
        const uint64_t want = (units + per_block - 1) / per_block;
        max_blocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 1), 1u << 30);
    }
    return enqueue(pl, d_descs, m, s, nullptr, 1, max_blocks, dsts);
}

uint32_t small_batch_grid(const ppc_plan* pl, uint32_t m, uint64_t bytes) {
    const ppc_batch_config& c = pl->cfg;
    const uint32_t g = (uint32_t)(c.blocks_per_cu * pl->cus);
    const uint64_t units = (uint64_t)m * (uint64_t)c.stream_weight + bytes / 16;
    const uint64_t per_block = kFreshUnitsPerWave * (uint64_t)(c.block_threads / kWave);
    const uint64_t want = std::max<uint64_t>((units + per_block - 1) / per_block, 1);
    return want < g ? (uint32_t)want : g;
}

int batch_zeroed(ppc_plan* pl, const ppc_desc* d_descs, uint32_t m, hipStream_t s,
                 uint64_t bytes, uint8_t* const* dsts) {
    if (!pl || !d_descs) return PPC_ERR_NULL;
    // (m <= kSmallBatch: d_descs may be pinned host memory, read once per block)
    if (m == 0) return PPC_OK;
    if (m > pl->max_streams) return PPC_ERR_ARG;
    if (m > kSmallBatch) return batch_fresh(pl, d_descs, m, s, bytes, dsts);
    const ppc_batch_config& c = pl->cfg;
    const uint32_t G = small_batch_grid(pl, m, bytes);
    uint64_t weight = (uint64_t)c.stream_weight;
    void* args[] = {(void*)&d_descs, (void*)&dsts, &m, &weight};
    PPC_HIP(hipLaunchKernel(small_kernel(c.depth, dsts != nullptr), dim3(G), dim3(c.block_threads),
                            args, 0, s));
    return PPC_OK;
}
}  // namespace ppc

extern "C" {

int ppc_plan_create(const ppc_workload_hint* hint, ppc_plan** out) {
    if (!hint || !out) return PPC_ERR_NULL;
    *out = nullptr;
    if (hint->max_streams == 0 || hint->max_streams > kMaxPlanStreams) return PPC_ERR_ARG;
    // the configuration a new plan starts from: the default, or the environment's
    ppc_batch_config initial = default_config();
    const EnvBatch& env = env_batch();
    if (env.set) {
        if (env.cfg.depth) initial.depth = env.cfg.depth;
        if (env.cfg.block_threads) initial.block_threads = env.cfg.block_threads;
        if (env.cfg.blocks_per_cu) initial.blocks_per_cu = env.cfg.blocks_per_cu;
        if (env.cfg.stream_weight) initial.stream_weight = env.cfg.stream_weight;
        if (env.bad || check_config(initial)) return PPC_ERR_ARG;
    }
    const DeviceFacts* dev = nullptr;
    int st = current_device(&dev);
    if (st) return st;
    ppc_plan* pl = new ppc_plan();
    pl->device = dev->device;
    pl->max_streams = hint->max_streams;
    pl->flags = hint->flags;
    pl->cus = dev->cus;
    pl->gmax = dev->cus * kMaxBlocksPerCu;
    memcpy(pl->arch, dev->arch, sizeof(pl->arch));
    pl->cfg = initial;
    const size_t cum_bytes = ((size_t)hint->max_streams + 1) * 8;
    const size_t first_bytes = (size_t)pl->gmax * 4;
    const size_t off_first = (cum_bytes + 255) & ~(size_t)255;
    const size_t off_rej = (off_first + first_bytes + 255) & ~(size_t)255;
    const size_t off_sink = off_rej + 256;
    const size_t chunks = ((size_t)hint->max_streams + kChunk - 1) / kChunk;
    const size_t off_part = off_sink + (size_t)pl->gmax * 32 * 8;
    const size_t off_part_bad = off_part + ((chunks * 8 + 255) & ~(size_t)255);
    const size_t total = off_part_bad + chunks * 4;
    hipError_t e = hipMalloc(&pl->scratch, total);
    if (e != hipSuccess) {
        delete pl;
        return fail_hip(e);
    }
    char* base = (char*)pl->scratch;
    pl->cum = (uint64_t*)base;
    pl->first = (uint32_t*)(base + off_first);
    pl->rejected = (uint32_t*)(base + off_rej);
    pl->sink = (unsigned long long*)(base + off_sink);
    pl->part = (uint64_t*)(base + off_part);
    pl->part_bad = (uint32_t*)(base + off_part_bad);
    e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(pl->scratch);
        delete pl;
        return fail_hip(e);
    }
    *out = pl;
    return PPC_OK;
}

int ppc_plan_destroy(ppc_plan* pl) {
    if (!pl) return PPC_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != pl->device) (void)hipSetDevice(pl->device);
    // Work enqueued with the plan reads its scratch (and may replay its graph): wait
    // for the device, so that dropping a plan early frees nothing still in use.
    (void)hipDeviceSynchronize();
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->scratch) (void)hipFree(pl->scratch);
    if (dev >= 0 && dev != pl->device) (void)hipSetDevice(dev);
    delete pl;
    return PPC_OK;
}

int pospopcnt_batch(ppc_plan* pl, const ppc_desc* d_descs, uint32_t m, ppc_stream stream) {
    if (!pl) return PPC_ERR_NULL;
    if (m == 0) return PPC_OK;
    if (!d_descs) return PPC_ERR_NULL;
    if ((uintptr_t)d_descs & 7u) return PPC_ERR_ALIGN;
    if (m > pl->max_streams) return PPC_ERR_ARG;
    int st = device_of(pl);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!(pl->flags & PPC_PLAN_GRAPH)) return enqueue(pl, d_descs, m, s, nullptr);
    if (!pl->exec || pl->g_descs != d_descs || pl->g_m != m || pl->g_version != pl->cfg_version) {
        if (pl->exec) {
            PPC_HIP(hipGraphExecDestroy(pl->exec));
            pl->exec = nullptr;
        }
        PPC_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
        const int est = enqueue(pl, d_descs, m, pl->cap_stream, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(pl->cap_stream, &g);
        if (est) {
            if (g) (void)hipGraphDestroy(g);
            return est;
        }
        if (ce != hipSuccess) return fail_hip(ce);
        const hipError_t ie = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            pl->exec = nullptr;
            return fail_hip(ie);
        }
        pl->g_descs = d_descs;
        pl->g_m = m;
        pl->g_version = pl->cfg_version;
    }
    PPC_HIP(hipGraphLaunch(pl->exec, s));
    return PPC_OK;
}

int pospopcnt_batch_static(const ppc_desc* d_descs, uint32_t m, const ppc_batch_config* config,
                           ppc_stream stream) {
    if (m == 0) return PPC_OK;
    if (!d_descs) return PPC_ERR_NULL;
    if ((uintptr_t)d_descs & 7u) return PPC_ERR_ALIGN;
    if (m > PPC_STATIC_MAX_STREAMS) return PPC_ERR_CAPACITY;
    const ppc_batch_config c = config ? *config : default_config();
    int st = check_config(c);
    if (st) return st;
    const DeviceFacts* dev = nullptr;
    if ((st = current_device(&dev))) return st;
    if ((int64_t)c.blocks_per_cu * dev->cus > (int64_t)kStaticMaxBlocks) return PPC_ERR_CAPACITY;
    char* base = nullptr;
    if ((st = static_scratch(dev->device, &base))) return st;
    const BatchScratch sc{(uint64_t*)(base + kStaticCumOff), (uint32_t*)(base + kStaticFirstOff),
                          (uint32_t*)(base + kStaticRejOff), (uint64_t*)(base + kStaticPartOff),
                          (uint32_t*)(base + kStaticPartBadOff)};
    return enqueue_with(sc, c, dev->cus, d_descs, m, (hipStream_t)stream, nullptr, 0, 0);
}

int ppc_plan_get_config(const ppc_plan* pl, ppc_batch_config* c) {
    if (!pl || !c) return PPC_ERR_NULL;
    *c = pl->cfg;
    return PPC_OK;
}

int ppc_plan_set_config(ppc_plan* pl, const ppc_batch_config* c) {
    if (!pl || !c) return PPC_ERR_NULL;
    int st = check_config(*c);
    if (st) return st;
    pl->cfg = *c;
    ++pl->cfg_version;
    return PPC_OK;
}

int ppc_plan_autotune(ppc_plan* pl, const ppc_desc* d_descs, uint32_t m, ppc_stream stream,
                      float* best_ms) {
    if (!pl) return PPC_ERR_NULL;
    if (m == 0) return PPC_OK;
    if (!d_descs) return PPC_ERR_NULL;
    if ((uintptr_t)d_descs & 7u) return PPC_ERR_ALIGN;
    if (m > pl->max_streams) return PPC_ERR_ARG;
    int st = device_of(pl);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    // Shallow circuits keep fewer bytes in flight per wave (4 dwords per lane per
    // tile at depth 4), so the axis of waves per CU reaches 16.
    std::vector<ppc_batch_config> cands;
    for (int depth : {4, 8, 16, 32}) {
        for (int bpc : {2, 3, 4, 6, 8, 12, 16})
            for (int weight : {1024, 2048, 4096, 8192}) cands.push_back({depth, 64, bpc, weight});
        for (int bpc : {1, 2, 3, 4})
            for (int weight : {2048, 4096}) cands.push_back({depth, 256, bpc, weight});
    }
    hipEvent_t e0, e1;
    PPC_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail_hip(he);
    }
    const ppc_batch_config saved = pl->cfg;
    // One timed launch of the plan as configured by c.
    auto timed = [&](const ppc_batch_config& c, float* t) -> int {
        pl->cfg = c;
        if ((he = hipEventRecord(e0, s)) != hipSuccess) return PPC_ERR_HIP;
        if (int r = enqueue(pl, d_descs, m, s, pl->sink)) return r;
        if ((he = hipEventRecord(e1, s)) != hipSuccess) return PPC_ERR_HIP;
        if ((he = hipEventSynchronize(e1)) != hipSuccess) return PPC_ERR_HIP;
        if ((he = hipEventElapsedTime(t, e0, e1)) != hipSuccess) return PPC_ERR_HIP;
        return PPC_OK;
    };
    auto median = [](std::vector<float> v) {
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
    };
    // Stage 1: every candidate, a warm-up launch and the median of 3.  Many shapes
    // land within the run-to-run noise of the best, so the smallest of these
    // medians favours a lucky one; stage 2 times the kTop fastest again, kReps
    // times each, taking the candidates in turn so that a drift of the clock or
    // of the memory rate reaches all of them alike, and keeps the lowest median.
    constexpr size_t kTop = 4;
    constexpr int kReps = 5;
    std::vector<std::pair<float, size_t>> first;
    int rc = PPC_OK;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        pl->cfg = cands[i];
        if ((rc = enqueue(pl, d_descs, m, s, pl->sink))) break;  // warm-up
        std::vector<float> ts(3);
        for (float& t : ts)
            if ((rc = timed(cands[i], &t))) break;
        if (!rc) first.push_back({median(ts), i});
    }
    ppc_batch_config best = saved;
    float best_t = INFINITY;
    if (!rc) {
        std::sort(first.begin(), first.end());
        const size_t top = std::min(kTop, first.size());
        std::vector<std::vector<float>> again(top);
        for (int r = 0; r < kReps && !rc; ++r)
            for (size_t j = 0; j < top && !rc; ++j) {
                float t = 0;
                if (!(rc = timed(cands[first[j].second], &t))) again[j].push_back(t);
            }
        for (size_t j = 0; j < top && !rc; ++j) {
            const float t = median(again[j]);
            if (t < best_t) {
                best_t = t;
                best = cands[first[j].second];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == PPC_ERR_HIP && he != hipSuccess) rc = fail_hip(he);
    pl->cfg = rc ? saved : best;
    ++pl->cfg_version;
    if (!rc && best_ms) *best_ms = best_t;
    return rc;
}

int ppc_plan_save(const ppc_plan* pl, const char* path) {
    if (!pl || !path) return PPC_ERR_NULL;
    FILE* f = fopen(path, "w");
    if (!f) return PPC_ERR_ARG;
    fprintf(f,
            "{\"arch\": \"%s\", \"depth\": %d, \"block_threads\": %d, \"blocks_per_cu\": %d, "
            "\"stream_weight\": %d}\n",
            pl->arch, pl->cfg.depth, pl->cfg.block_threads, pl->cfg.blocks_per_cu,
            pl->cfg.stream_weight);
    return fclose(f) == 0 ? PPC_OK : PPC_ERR_ARG;
}

static bool json_int(const char* text, const char* key, int* out) {
    char pat[64];
    snprintf(pat, sizeof(pat), "\"%s\"", key);
    const char* p = strstr(text, pat);
    if (!p) return false;
    p = strchr(p + strlen(pat), ':');
    return p && sscanf(p + 1, "%d", out) == 1;
}

int ppc_plan_load(ppc_plan* pl, const char* path) {
    if (!pl || !path) return PPC_ERR_NULL;
    FILE* f = fopen(path, "r");
    if (!f) return PPC_ERR_ARG;
    char text[1024] = {0};
    const size_t got = fread(text, 1, sizeof(text) - 1, f);
    fclose(f);
    text[got] = 0;
    const char* a = strstr(text, "\"arch\"");
    char arch[64] = {0};
    if (!a || sscanf(a, "\"arch\" : \"%63[^\"]\"", arch) != 1) {
        if (!a || sscanf(a, "\"arch\": \"%63[^\"]\"", arch) != 1) return PPC_ERR_ARG;
    }
    ppc_batch_config c{};
    if (!json_int(text, "depth", &c.depth) || !json_int(text, "block_threads", &c.block_threads) ||
        !json_int(text, "blocks_per_cu", &c.blocks_per_cu) ||
        !json_int(text, "stream_weight", &c.stream_weight))
        return PPC_ERR_ARG;
    if (strcmp(arch, pl->arch) != 0) return PPC_ERR_STATE;
    if (check_config(c)) return PPC_ERR_ARG;
    pl->cfg = c;
    ++pl->cfg_version;
    return PPC_OK;
}

// ---- keyed cache of tuned configurations: one JSON object per line

static int floor_log2(uint64_t x) {
    int r = -1;
    while (x) {
        x >>= 1;
        ++r;
    }
    return r;
}

struct CacheKey {
    char arch[64];
    int cus, streams_log2, bytes_log2;
};

static bool parse_entry(const char* line, CacheKey* key, ppc_batch_config* c) {
    const char* a = strstr(line, "\"arch\"");
    if (!a || sscanf(a, "\"arch\": \"%63[^\"]\"", key->arch) != 1) return false;
    return json_int(line, "cus", &key->cus) && json_int(line, "streams_log2", &key->streams_log2) &&
           json_int(line, "bytes_log2", &key->bytes_log2) && json_int(line, "depth", &c->depth) &&
           json_int(line, "block_threads", &c->block_threads) &&
           json_int(line, "blocks_per_cu", &c->blocks_per_cu) &&
           json_int(line, "stream_weight", &c->stream_weight);
}

static bool same_key(const CacheKey& a, const CacheKey& b) {
    return !strcmp(a.arch, b.arch) && a.cus == b.cus && a.streams_log2 == b.streams_log2 &&
           a.bytes_log2 == b.bytes_log2;
}

static CacheKey key_of(const ppc_plan* pl, uint32_t m, uint64_t bytes) {
    CacheKey k;
    memset(&k, 0, sizeof(k));
    memcpy(k.arch, pl->arch, sizeof(k.arch));
    k.arch[sizeof(k.arch) - 1] = 0;
    k.cus = pl->cus;
    k.streams_log2 = floor_log2(m);
    k.bytes_log2 = floor_log2(bytes);
    return k;
}

// Reads every line of a cache file; a missing file is an empty cache.  false if a
// line does not parse.
static bool read_cache(const char* path, std::vector<std::pair<CacheKey, ppc_batch_config>>* out) {
    FILE* f = fopen(path, "r");
    if (!f) return true;
    char line[1024];
    bool ok = true;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '\n' || line[0] == 0) continue;
        CacheKey k;
        ppc_batch_config c{};
        if (!parse_entry(line, &k, &c)) {
            ok = false;
            break;
        }
        out->push_back({k, c});
    }
    fclose(f);
    return ok;
}

int ppc_plan_cache_put(const ppc_plan* pl, const char* path, uint32_t m, uint64_t bytes) {
    if (!pl || !path) return PPC_ERR_NULL;
    if (m == 0 || bytes == 0) return PPC_ERR_ARG;
    std::vector<std::pair<CacheKey, ppc_batch_config>> entries;
    if (!read_cache(path, &entries)) return PPC_ERR_ARG;
    const CacheKey key = key_of(pl, m, bytes);
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return PPC_ERR_ARG;
    auto write = [&](const CacheKey& k, const ppc_batch_config& c) {
        fprintf(f,
                "{\"arch\": \"%s\", \"cus\": %d, \"streams_log2\": %d, \"bytes_log2\": %d, "
                "\"depth\": %d, \"block_threads\": %d, \"blocks_per_cu\": %d, "
                "\"stream_weight\": %d}\n",
                k.arch, k.cus, k.streams_log2, k.bytes_log2, c.depth, c.block_threads,
                c.blocks_per_cu, c.stream_weight);
    };
    for (const auto& e : entries)
        if (!same_key(e.first, key)) write(e.first, e.second);
    write(key, pl->cfg);
    if (fclose(f) != 0) return PPC_ERR_ARG;
    return rename(tmp.c_str(), path) == 0 ? PPC_OK : PPC_ERR_ARG;
}

int ppc_plan_cache_get(ppc_plan* pl, const char* path, uint32_t m, uint64_t bytes) {
    if (!pl || !path) return PPC_ERR_NULL;
    if (m == 0 || bytes == 0) return PPC_ERR_ARG;
    std::vector<std::pair<CacheKey, ppc_batch_config>> entries;
    if (!read_cache(path, &entries)) return PPC_ERR_ARG;
    const CacheKey key = key_of(pl, m, bytes);
    for (auto it = entries.rbegin(); it != entries.rend(); ++it) {
        if (!same_key(it->first, key)) continue;
        if (check_config(it->second)) return PPC_ERR_ARG;
        pl->cfg = it->second;
        ++pl->cfg_version;
        return PPC_OK;
    }
    return PPC_ERR_STATE;
}

int ppc_plan_rejected(ppc_plan* pl, ppc_stream stream, uint32_t* out) {
    if (!pl || !out) return PPC_ERR_NULL;
    int st = device_of(pl);
    if (st) return st;
    PPC_HIP(hipMemcpyAsync(out, pl->rejected, 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
    PPC_HIP(hipStreamSynchronize((hipStream_t)stream));
    return PPC_OK;
}

int pospopcnt_each(const ppc_desc* h, uint32_t m, ppc_stream stream) {
    if (m == 0) return PPC_OK;
    if (!h) return PPC_ERR_NULL;
    for (uint32_t i = 0; i < m; ++i) {
        if (h[i].reserved) return PPC_ERR_ARG;
        if (h[i].k == 64) return PPC_ERR_WIDTH;  // as in the batched form
        uint64_t nb = 0;
        int st = check_stream_args(h[i].ptr, h[i].n, (int)h[i].k, h[i].counts, &nb);
        if (st) return st;
    }
    for (uint32_t i = 0; i < m; ++i) {
        int st = launch_stream(h[i].ptr, h[i].n, (int)h[i].k, h[i].counts, stream, nullptr);
        if (st) return st;
    }
    return PPC_OK;
}

}  // extern "C"
