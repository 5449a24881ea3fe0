// ppc_onehot.hip -- histogram of categorical ids as the positional population
// count of their one-hot codes, without writing the codes anywhere.
//
// The paper's motivating use (Sec. 1, Table 1): with `bins` categories, category
// c is bit c of a bins-bit one-hot word, and the positional population count of
// the encoded stream is the frequency histogram.  Here each lane loads raw ids
// (u8 or u16) with the same nontemporal dwordx4 tiles as the counting kernel,
// expands every id into its one-hot dword in registers (1 << id, or nothing for
// an id >= bins, which is tallied apart), and feeds the one-hot dwords to the
// Harley-Seal circuit of Sec. 2: 64 u8 ids (or 32 u16 ids) per lane per tile make
// one 64- (32-) input circuit, whose carry is counted per category class as in
// the counting kernel.  Head and tail ids outside the 16-byte aligned body are
// expanded one per lane by the first wave; padding never becomes an id.
#include "ppc_device.h"
#include "ppc_internal.h"

namespace ppc {

constexpr int kOnehotThreads = 256;

// One-hot dwords of the ids in dword x (4 u8 ids or 2 u16 ids, low id first).
// Ids >= C have no code; they add to `other`.  valid = false: x holds no ids.
template <int C, int IDB>
__device__ __forceinline__ void expand(uint32_t* o, uint32_t x, uint32_t& other, bool valid) {
#pragma unroll
    for (int i = 0; i < 4 / IDB; ++i) {
        const uint32_t id = IDB == 1 ? (x >> (8 * i)) & 0xFFu : (x >> (16 * i)) & 0xFFFFu;
        const bool code = valid && id < (uint32_t)C;
        o[i] = code ? (1u << id) : 0u;
        other += (valid && !code) ? 1u : 0u;
    }
}

template <int C, int IDB, int U, int LOGD>
__device__ __forceinline__ void onehot_step(uint32_t (&B)[LOGD], uint32_t (&cnt)[C],
                                            uint32_t& other, const u32x4 (&v)[U],
                                            const bool (&valid)[U]) {
    constexpr int PER = 4 / IDB;
    static_assert(4 * U * PER == (1 << LOGD), "one circuit per tile");
    uint32_t d[4 * U * PER];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        expand<C, IDB>(d + (4 * j + 0) * PER, v[j].x, other, valid[j]);
        expand<C, IDB>(d + (4 * j + 1) * PER, v[j].y, other, valid[j]);
        expand<C, IDB>(d + (4 * j + 2) * PER, v[j].z, other, valid[j]);
        expand<C, IDB>(d + (4 * j + 3) * PER, v[j].w, other, valid[j]);
    }
    count_classes<C>(cnt, Circuit<LOGD>::run(B, d));
}

// The id at head or tail position `lane` of the first wave: lanes 0..15 take
// head ids, lanes 16..31 tail ids.  u16 ids are 2-byte aligned, so the head and
// tail hold whole ids.
template <int C, int IDB>
__device__ __forceinline__ uint32_t edge_onehot(const Edges& e, int lane, uint32_t& other) {
    const uint8_t* p = nullptr;
    if (lane < 16) {
        if ((uint32_t)(lane * IDB) < e.head_len) p = e.head + lane * IDB;
    } else if (lane < 32) {
        if ((uint32_t)((lane - 16) * IDB) < e.tail_len) p = e.tail + (lane - 16) * IDB;
    }
    if (!p) return 0u;
    const uint32_t id = IDB == 1 ? (uint32_t)p[0] : (uint32_t)p[0] | ((uint32_t)p[1] << 8);
    if (id < (uint32_t)C) return 1u << id;
    ++other;
    return 0u;
}

template <int C, int IDB>
__global__ void __launch_bounds__(kOnehotThreads)
onehot_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges,
              unsigned long long* __restrict__ counts) {
    constexpr int U = 4;
    constexpr int LOGD = IDB == 1 ? 6 : 5;  // 64 u8 or 32 u16 ids per lane per tile
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t full = units / TILE;

    uint32_t B[LOGD], cnt[C], other = 0;
#pragma unroll
    for (int j = 0; j < LOGD; ++j) B[j] = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) cnt[i] = 0;
    const bool all[U] = {true, true, true, true};
    walk_tiles<U>(body, full, gw, nw, lane, [&](const u32x4(&v)[U]) {
        onehot_step<C, IDB, U, LOGD>(B, cnt, other, v, all);
    });
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 t[U];
        load_tile_masked<U>(t, body + full * TILE + lane, lane, rem);
        bool valid[U];
#pragma unroll
        for (int j = 0; j < U; ++j) valid[j] = (uint64_t)(j * kWave + lane) < rem;
        onehot_step<C, IDB, U, LOGD>(B, cnt, other, t, valid);
    }
    const uint32_t e = (blockIdx.x == 0 && wave == 0) ? edge_onehot<C, IDB>(edges, lane, other) : 0u;

    uint32_t tot[C];
    lane_totals<C, LOGD>(tot, cnt, B, e);
    const uint32_t v = wave_reduce_scatter<C>(tot, lane);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) other += (uint32_t)__shfl_xor((int)other, o, kWave);
    __shared__ uint32_t red[kOnehotThreads / kWave][C];
    __shared__ uint32_t red_other[kOnehotThreads / kWave];
    constexpr int G = kWave / C;
    if (lane % G == 0) red[wave][lane / G] = v;
    if (lane == 0) red_other[wave] = other;
    __syncthreads();
    block_flush<C>(red, wpb, C, 0u, counts);
    if (threadIdx.x == C) {
        unsigned long long s = 0;
        for (int w = 0; w < wpb; ++w) s += red_other[w];
        if (s) atomicAdd(counts + C, s);
    }
}

using OnehotKernel = void (*)(const u32x4*, uint64_t, Edges, unsigned long long*);

static const void* onehot_of(int bins, int id_bytes) {
    static OnehotKernel table[2][3] = {
        {onehot_kernel<8, 1>, onehot_kernel<16, 1>, onehot_kernel<32, 1>},
        {onehot_kernel<8, 2>, onehot_kernel<16, 2>, onehot_kernel<32, 2>},
    };
    return (const void*)table[id_bytes - 1][bins == 8 ? 0 : bins == 16 ? 1 : 2];
}

static int launch_histogram(const void* ids, uint64_t n, int id_bytes, int bins,
                            uint64_t* counts, ppc_stream stream, const ppc_launch_config* cfg) {
    if (id_bytes != 1 && id_bytes != 2) return PPC_ERR_ARG;
    if (bins != 8 && bins != 16 && bins != 32) return PPC_ERR_WIDTH;
    if (n == 0) return PPC_OK;
    if (n > UINT64_MAX / (uint64_t)id_bytes) return PPC_ERR_RANGE;
    const uint64_t nbytes = n * (uint64_t)id_bytes;
    if (!ids || !counts) return PPC_ERR_NULL;
    if ((uintptr_t)counts & 7u) return PPC_ERR_ALIGN;
    if (id_bytes == 2 && ((uintptr_t)ids & 1u)) return PPC_ERR_ALIGN;
    const uintptr_t p = (uintptr_t)ids;
    if (p + nbytes < p) return PPC_ERR_RANGE;
    const uintptr_t c0 = (uintptr_t)counts, c1 = c0 + 8u * (uintptr_t)(bins + 1);
    if (c0 < p + nbytes && p < c1) return PPC_ERR_OVERLAP;
    ppc_launch_config c = {};
    if (cfg) c = *cfg;
    if (c.variant != PPC_VARIANT_CSA || (c.depth != 0)) return PPC_ERR_ARG;
    const int threads = c.block_threads ? c.block_threads : kOnehotThreads;
    if (threads < kWave || threads > kOnehotThreads || threads % kWave) return PPC_ERR_ARG;
    if (c.blocks_per_cu < 0 || c.grid < 0) return PPC_ERR_ARG;
    const DeviceFacts* dev = nullptr;
    int st = current_device(&dev);
    if (st) return st;
    const Split s = split_stream(ids, nbytes, 8);
    const int wpb = threads / kWave;
    const uint64_t tiles = (s.units + kWave * 4 - 1) / (kWave * 4);
    uint64_t need = (tiles + wpb - 1) / wpb;
    if (need == 0) need = 1;
    int64_t grid;
    if (c.grid > 0) {
        grid = c.grid;
    } else {
        // More resident waves than the counting kernel: each id costs an
        // expansion on top of its share of the circuit, so there is more
        // arithmetic to overlap with the loads.
        const int bpc = c.blocks_per_cu ? c.blocks_per_cu : 2;
        grid = (int64_t)bpc * dev->cus;
        if ((uint64_t)grid > need) grid = (int64_t)need;
    }
    const int64_t min_grid = (int64_t)(nbytes >> 31) + 1;  // per-block totals below 2^32
    if (grid < min_grid) grid = min_grid;
    if (grid > 0x7fffffff) return PPC_ERR_ARG;
    Edges e{s.head, s.tail, s.head_len, s.tail_len};
    const u32x4* body = (const u32x4*)s.body;
    uint64_t units = s.units;
    unsigned long long* cp = (unsigned long long*)counts;
    void* args[] = {&body, &units, &e, &cp};
    PPC_HIP(hipLaunchKernel(onehot_of(bins, id_bytes), dim3((uint32_t)grid), dim3(threads), args,
                            0, (hipStream_t)stream));
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

extern "C" {

int ppc_histogram_u8(const void* ids, uint64_t n, uint32_t bins, uint64_t* counts,
                     ppc_stream stream) {
    return launch_histogram(ids, n, 1, (int)bins, counts, stream, nullptr);
}

int ppc_histogram_u16(const void* ids, uint64_t n, uint32_t bins, uint64_t* counts,
                      ppc_stream stream) {
    return launch_histogram(ids, n, 2, (int)bins, counts, stream, nullptr);
}

int ppc_histogram_ex(const void* ids, uint64_t n, int id_bytes, uint32_t bins, uint64_t* counts,
                     ppc_stream stream, const ppc_launch_config* config) {
    return launch_histogram(ids, n, id_bytes, (int)bins, counts, stream, config);
}

}  // extern "C"
