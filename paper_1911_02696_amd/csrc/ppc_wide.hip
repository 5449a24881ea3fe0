// ppc_wide.hip -- words wider than 32 bits (Sec. 4: the method generalises to
// wider words, and wider words can be held as several streams of 16-bit words).
//
// k = 64, one stream of 64-bit words.  Give the dword at address A (A a multiple
// of 4) the parity q = (A/4) mod 2; in a stream that starts at a multiple of 8,
// dwords of parity 0 hold word bits 0..31 and dwords of parity 1 bits 32..63.
// In the 16-byte aligned body the parities alternate: x and z of every dwordx4
// load have parity 0, y and w parity 1.  Each lane therefore runs two
// Harley-Seal circuits of Sec. 2 per tile, one over each parity, and counts 64
// classes: class 32q + i is bit i of a dword of parity q.  For a stream that
// starts at ptr with r = ptr mod 8, that class is word bit (32q + i - 8r) mod 64,
// the same rotation at the flush as for the narrower widths.  Tile carries go
// through the cross-tile levels of ppc_tree.h, so the 32-class count of a carry
// runs once every 2^E tiles.
//
// k = 16m as m planes of 16-bit words: one launch whose grid has one row of
// blocks per plane (blockIdx.y); each row counts its plane exactly like the
// single-stream pospopcnt16 kernel (count_stream) into counters 16j .. 16j+15.
#include "ppc_device.h"
#include "ppc_internal.h"
#include "ppc_tree.h"

namespace ppc {

constexpr int kWideThreads = 256;
constexpr int kWideWaves = kWideThreads / kWave;

// The edge byte of `lane` (lanes 0..14 head, 16..30 tail) at its place in its
// aligned dword, and that dword's parity (A/4) mod 2.
__device__ __forceinline__ uint32_t edge_dword_q(const Edges& e, int lane, uint32_t* q) {
    const uint8_t* p = nullptr;
    if (lane < 16) {
        if ((uint32_t)lane < e.head_len) p = e.head + lane;
    } else if (lane < 32) {
        if ((uint32_t)(lane - 16) < e.tail_len) p = e.tail + (lane - 16);
    }
    *q = 0;
    if (!p) return 0u;
    *q = (uint32_t)(((uintptr_t)p >> 2) & 1u);
    return (uint32_t)(*p) << (8u * (uint32_t)((uintptr_t)p & 3u));
}

// LOGH: log2 of the dwords of one parity per lane and tile (a tile is 2^(LOGH+1)
// dwords per lane, 2^(LOGH-1) dwordx4 loads).  E: cross-tile levels per parity.
template <int LOGH, int E>
__global__ void __launch_bounds__(kWideThreads)
wide64_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges, uint32_t rot,
              unsigned long long* __restrict__ counts) {
    constexpr int U = (1 << (LOGH + 1)) / 4;
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t full = units / TILE;

    uint32_t Blo[LOGH], Bhi[LOGH];
#pragma unroll
    for (int j = 0; j < LOGH; ++j) Blo[j] = Bhi[j] = 0;
    TileTree<32, LOGH, E> lo, hi;
    lo.init();
    hi.init();
    auto step = [&](const u32x4(&v)[U]) {
        uint32_t de[2 * U], dq[2 * U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            de[2 * j] = v[j].x;
            de[2 * j + 1] = v[j].z;
            dq[2 * j] = v[j].y;
            dq[2 * j + 1] = v[j].w;
        }
        lo.add(Circuit<LOGH>::run(Blo, de));
        hi.add(Circuit<LOGH>::run(Bhi, dq));
    };
    walk_tiles<U>(body, full, gw, nw, lane, step);
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 a[U];
        load_tile_masked<U>(a, body + full * TILE + lane, lane, rem);
        step(a);
    }

    uint32_t q = 0;
    const uint32_t e = (blockIdx.x == 0 && wave == 0) ? edge_dword_q(edges, lane, &q) : 0u;
    uint32_t tlo[32], thi[32], tot[64];
    lo.totals(tlo, Blo, q ? 0u : e);
    hi.totals(thi, Bhi, q ? e : 0u);
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        tot[i] = tlo[i];
        tot[32 + i] = thi[i];
    }
    const uint32_t v = wave_reduce_scatter<64>(tot, lane);
    __shared__ uint32_t red[kWideWaves][64];
    red[wave][lane] = v;
    __syncthreads();
    block_flush<64>(red, wpb, 64, rot, counts);
}

// Up to PPC_MAX_PLANES planes per launch, passed by value in the kernel arguments.
struct PlaneArgs {
    const u32x4* body;
    uint64_t units;
    Edges edges;
    unsigned long long* counts;
    uint32_t rot;
    uint32_t unused;
};
struct PlaneTable {
    PlaneArgs p[PPC_MAX_PLANES];
};

template <int LOGD>
__global__ void __launch_bounds__(kWideThreads)
planes16_kernel(PlaneTable t) {
    __shared__ uint32_t red[kWideWaves][16];
    const PlaneArgs& a = t.p[blockIdx.y];
    count_stream<16, LOGD>(a.body, a.units, a.edges, 16, a.rot, a.counts, blockIdx.x, gridDim.x,
                           red);
}

using Wide64Kernel = void (*)(const u32x4*, uint64_t, Edges, uint32_t, unsigned long long*);
using PlanesKernel = void (*)(PlaneTable);

// Circuit inputs per lane and tile, both parities: 4, 8, 16 (default) or 32 dwords;
// the cross-tile levels make every depth count classes once per 64 dwords of a
// parity.
static const void* wide64_of(int depth) {
    static Wide64Kernel table[4] = {wide64_kernel<1, 5>, wide64_kernel<2, 4>, wide64_kernel<3, 3>,
                                    wide64_kernel<4, 2>};
    return (const void*)table[logd_of_depth(depth) - 2];
}

static const void* planes_of(int depth) {
    static PlanesKernel table[4] = {planes16_kernel<2>, planes16_kernel<3>, planes16_kernel<4>,
                                    planes16_kernel<5>};
    return (const void*)table[logd_of_depth(depth) - 2];
}

// Shared launch-shape rules: the configuration's block size and blocks per CU,
// or the defaults (few waves per CU, as for the counting kernel).
struct WideShape {
    int depth, threads, bpc;
};

static int wide_shape(const ppc_launch_config* cfg, int def_threads, int def_bpc, WideShape* out) {
    ppc_launch_config c = {};
    if (cfg) c = *cfg;
    if (c.variant != PPC_VARIANT_CSA) return PPC_ERR_ARG;
    const int depth = c.depth ? c.depth : 16;
    if (logd_of_depth(depth) < 0) return PPC_ERR_ARG;
    const int threads = c.block_threads ? c.block_threads : def_threads;
    if (threads < kWave || threads > kWideThreads || threads % kWave) return PPC_ERR_ARG;
    if (c.blocks_per_cu < 0 || c.grid < 0) return PPC_ERR_ARG;
    out->depth = depth;
    out->threads = threads;
    out->bpc = c.blocks_per_cu ? c.blocks_per_cu : def_bpc;
    return PPC_OK;
}

int launch_wide64(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream,
                  const ppc_launch_config* cfg) {
    uint64_t nbytes = 0;
    int st = check_stream_args(ptr, n, 64, counts, &nbytes);
    if (st != PPC_OK || nbytes == 0) return st;
    WideShape sh;
    if ((st = wide_shape(cfg, 256, 1, &sh))) return st;
    const DeviceFacts* dev = nullptr;
    if ((st = current_device(&dev))) return st;
    const Split s = split_stream(ptr, nbytes, 64);
    const int wpb = sh.threads / kWave;
    const uint64_t tile_units = (uint64_t)kWave * (uint64_t)(sh.depth / 4);
    const uint64_t tiles = (s.units + tile_units - 1) / tile_units;
    uint64_t need = blocks_needed(tiles, wpb);
    if (need == 0) need = 1;
    int64_t grid = (cfg && cfg->grid > 0) ? cfg->grid : (int64_t)sh.bpc * dev->cus;
    if (!(cfg && cfg->grid > 0) && (uint64_t)grid > need) grid = (int64_t)need;
    // Every block's per-class total stays below 2^32 (a class takes at most one
    // bit per 8 input bytes; the bound below is the narrower kernels' one).
    const int64_t min_grid = (int64_t)(nbytes >> 31) + 1;
    if (grid < min_grid) grid = min_grid;
    if (grid > 0x7fffffff) return PPC_ERR_ARG;
    Edges e{s.head, s.tail, s.head_len, s.tail_len};
    const u32x4* body = (const u32x4*)s.body;
    uint64_t units = s.units;
    uint32_t rot = s.rot;
    unsigned long long* cp = (unsigned long long*)counts;
    void* args[] = {&body, &units, &e, &rot, &cp};
    PPC_HIP(hipLaunchKernel(wide64_of(sh.depth), dim3((uint32_t)grid), dim3(sh.threads), args, 0,
                            (hipStream_t)stream));
    return PPC_OK;
}

static int launch_planes16(const void* const* planes, uint32_t m, uint64_t n, uint64_t* counts,
                           ppc_stream stream, const ppc_launch_config* cfg) {
    if (m < 1 || m > PPC_MAX_PLANES) return PPC_ERR_ARG;
    if (n == 0) return PPC_OK;
    if (!planes || !counts) return PPC_ERR_NULL;
    if ((uintptr_t)counts & 7u) return PPC_ERR_ALIGN;
    if (n > UINT64_MAX / 2) return PPC_ERR_RANGE;
    const uint64_t nbytes = 2 * n;
    const uintptr_t c0 = (uintptr_t)counts, c1 = c0 + 8u * 16u * (uintptr_t)m;
    for (uint32_t j = 0; j < m; ++j) {
        const uintptr_t p = (uintptr_t)planes[j];
        if (!p) return PPC_ERR_NULL;
        if (p + nbytes < p) return PPC_ERR_RANGE;
        if (c0 < p + nbytes && p < c1) return PPC_ERR_OVERLAP;
    }
    WideShape sh;
    int st = wide_shape(cfg, 256, 1, &sh);
    if (st) return st;
    const DeviceFacts* dev = nullptr;
    if ((st = current_device(&dev))) return st;
    PlaneTable t = {};
    uint64_t units_max = 0;
    for (uint32_t j = 0; j < m; ++j) {
        const Split s = split_stream(planes[j], nbytes, 16);
        t.p[j].body = (const u32x4*)s.body;
        t.p[j].units = s.units;
        t.p[j].edges = Edges{s.head, s.tail, s.head_len, s.tail_len};
        t.p[j].counts = (unsigned long long*)counts + 16u * j;
        t.p[j].rot = s.rot;
        if (s.units > units_max) units_max = s.units;
    }
    // The chip's blocks are shared out over the planes (all of a length).
    const int wpb = sh.threads / kWave;
    const uint64_t tile_units = (uint64_t)kWave * (uint64_t)(sh.depth / 4);
    uint64_t need = blocks_needed((units_max + tile_units - 1) / tile_units, wpb);
    if (need == 0) need = 1;
    int64_t per;
    if (cfg && cfg->grid > 0) {
        per = cfg->grid;
    } else {
        per = ((int64_t)sh.bpc * dev->cus + m - 1) / m;
        if ((uint64_t)per > need) per = (int64_t)need;
    }
    const int64_t min_grid = (int64_t)(nbytes >> 31) + 1;
    if (per < min_grid) per = min_grid;
    if (per > 0x7fffffff) return PPC_ERR_ARG;
    void* args[] = {&t};
    PPC_HIP(hipLaunchKernel(planes_of(sh.depth), dim3((uint32_t)per, m), dim3(sh.threads), args, 0,
                            (hipStream_t)stream));
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

extern "C" {

int pospopcnt_u64(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream) {
    return launch_wide64(ptr, n, counts, stream, nullptr);
}

int pospopcnt_planes16(const void* const* planes, uint32_t m, uint64_t n, uint64_t* counts,
                       ppc_stream stream) {
    return launch_planes16(planes, m, n, counts, stream, nullptr);
}

int pospopcnt_planes16_ex(const void* const* planes, uint32_t m, uint64_t n, uint64_t* counts,
                          ppc_stream stream, const ppc_launch_config* config) {
    return launch_planes16(planes, m, n, counts, stream, config);
}

}  // extern "C"
