// ppc_single.hip -- single-stream positional population count on gfx950.
//
// Decomposition of a stream of nbytes at byte address ptr (see split_stream):
// up to 15 head bytes before the first 16-byte boundary, a 16-byte aligned body
// read with dwordx4 loads, up to 15 tail bytes.  Head and tail bytes are counted
// as zero-padded partial dwords by 31 lanes of the first wave; the body by the
// whole grid.  Bit positions are counted per dword-bit class and rotated into
// word positions at the flush (ppc_device.h), so every start address takes the
// same path (the paper handles only whole 256-byte blocks in SIMD and leaves the
// rest to scalar code, end of Sec. 4.1).
//
// CSA kernel (Sec. 4.1 on a GPU lane instead of an AVX-512 register):
//   * a wave tile is 64 lanes x U dwordx4 loads, each load instruction reading
//     1 KiB of consecutive bytes; waves walk tiles grid-stride, two tiles in
//     flight per wave (the next tile is loaded before the current is reduced);
//   * each lane feeds its 4U = 2^LOGD dwords through the Harley-Seal circuit of
//     Sec. 2 (2^LOGD - 1 CSAs, two bitop3 each), keeping running planes B[0 ..
//     LOGD-1] in registers;
//   * the carry plane (weight 2^LOGD, deferred) is counted per class with AND +
//     popcount-accumulate into per-lane 32-bit counters (Fig. 6's role);
//   * at the end each lane adds its planes with weights 1, 2, 4, ... (Sec. 4.1),
//     the wave reduce-scatters its counters, the block sums its waves in LDS and
//     adds into counts with one 64-bit atomic per word position.
// Ballot kernel (transposition across the wave instead of per-lane counters):
//   for every dword bit i, a wave-wide ballot gathers bit i of 64 dwords into a
//   64-bit mask whose population count is added to a wave-uniform counter.
// Hybrid kernel: the CSA kernel's circuit, with each carry plane counted by the
//   ballot transposition instead of per-lane class counters (a carry is one
//   dword in 2^LOGD, so the 32 ballots per carry cost 32 / 2^LOGD per dword).
// Read-ceiling kernel: the CSA kernel's loads, tiling and grid with the
// arithmetic replaced by an XOR; it bounds what any counting kernel can reach.
#include <atomic>
#include <mutex>

#include "ppc_device.h"
#include "ppc_internal.h"

namespace ppc {

constexpr int kMaxThreads = 256;
constexpr int kMaxWaves = kMaxThreads / kWave;

template <int C, int LOGD>
__global__ void __launch_bounds__(kMaxThreads)
csa_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges, int k, uint32_t rot,
           unsigned long long* __restrict__ counts) {
    __shared__ uint32_t red[kMaxWaves][C];
    count_stream<C, LOGD>(body, units, edges, k, rot, counts, blockIdx.x, gridDim.x, red);
}

template <int C>
__device__ __forceinline__ void ballot_count(uint32_t (&acc)[C], uint32_t x) {
#pragma unroll
    for (int i = 0; i < 32; ++i)
        acc[i % C] += (uint32_t)__popcll(__ballot((x >> i) & 1u));
}

template <int C>
__global__ void __launch_bounds__(kMaxThreads)
ballot_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges, int k, uint32_t rot,
              unsigned long long* __restrict__ counts) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t tiles = (units + kWave - 1) / kWave;

    uint32_t acc[C];
#pragma unroll
    for (int i = 0; i < C; ++i) acc[i] = 0;
    for (uint64_t t = gw; t < tiles; t += nw) {
        const uint64_t u = t * kWave + lane;
        const u32x4 v = u < units ? stream_load(body + u) : u32x4{0u, 0u, 0u, 0u};
        ballot_count<C>(acc, v.x);
        ballot_count<C>(acc, v.y);
        ballot_count<C>(acc, v.z);
        ballot_count<C>(acc, v.w);
    }
    if (blockIdx.x == 0 && wave == 0) ballot_count<C>(acc, edge_dword(edges, lane));

    __shared__ uint32_t red[kMaxWaves][C];
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < C; ++i) red[wave][i] = acc[i];
    }
    __syncthreads();
    block_flush<C>(red, wpb, k, rot, counts);
}

template <int C, int LOGD>
__global__ void __launch_bounds__(kMaxThreads)
hybrid_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges, int k, uint32_t rot,
              unsigned long long* __restrict__ counts) {
    constexpr int U = (1 << LOGD) / 4;
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t full = units / TILE;

    // B: running planes per lane; carries: the wave's carry bits per class
    // (wave-uniform), weight 2^LOGD deferred
    uint32_t B[LOGD], carries[C];
#pragma unroll
    for (int j = 0; j < LOGD; ++j) B[j] = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) carries[i] = 0;
    auto step = [&](const u32x4(&v)[U]) {
        uint32_t d[4 * U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            d[4 * j + 0] = v[j].x;
            d[4 * j + 1] = v[j].y;
            d[4 * j + 2] = v[j].z;
            d[4 * j + 3] = v[j].w;
        }
        ballot_count<C>(carries, Circuit<LOGD>::run(B, d));
    };
    walk_tiles<U>(body, full, gw, nw, lane, step);
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 a[U];
        load_tile_masked<U>(a, body + full * TILE + lane, lane, rem);
        step(a);
    }
    const uint32_t e = (blockIdx.x == 0 && wave == 0) ? edge_dword(edges, lane) : 0u;

    // the lane's planes and edge dword, plus (once per wave, in lane 0) the carries
    uint32_t none[C], tot[C];
#pragma unroll
    for (int i = 0; i < C; ++i) none[i] = 0;
    lane_totals<C, LOGD>(tot, none, B, e);
#pragma unroll
    for (int i = 0; i < C; ++i) tot[i] += lane == 0 ? carries[i] << LOGD : 0u;
    const uint32_t v = wave_reduce_scatter<C>(tot, lane);
    __shared__ uint32_t red[kMaxWaves][C];
    constexpr int G = kWave / C;
    if (lane % G == 0) red[wave][lane / G] = v;
    __syncthreads();
    block_flush<C>(red, wpb, k, rot, counts);
}

template <int LOGD>
__global__ void __launch_bounds__(kMaxThreads)
ceiling_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges,
               unsigned long long* __restrict__ sink) {
    constexpr int U = (1 << LOGD) / 4;
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t full = units / TILE;

    uint32_t acc = 0;
    auto fold = [&](const u32x4(&v)[U]) {
#pragma unroll
        for (int j = 0; j < U; ++j) acc ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
    };
    walk_tiles<U>(body, full, gw, nw, lane, fold);
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 a[U];
        load_tile_masked<U>(a, body + full * TILE + lane, lane, rem);
        fold(a);
    }
    if (blockIdx.x == 0 && wave == 0) acc ^= edge_dword(edges, lane);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, kWave);
    __shared__ uint32_t red[kMaxWaves];
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = 0;
        for (int w = 0; w < wpb; ++w) x ^= red[w];
        if (x) atomicXor(sink, (unsigned long long)x);
    }
}

// ------------------------------------------------------------------ host side

using StreamKernel = void (*)(const u32x4*, uint64_t, Edges, int, uint32_t, unsigned long long*);
using CeilKernel = void (*)(const u32x4*, uint64_t, Edges, unsigned long long*);

static int class_index(int k) { return k == 8 ? 0 : k == 16 ? 1 : 2; }

// Circuits of 4, 8, 16 and 32 dwords per lane per step (LOGD 2 .. 5): the GPU
// counterparts of the 256 B, 512 B and 1 kB circuits of Sec. 4.1 (3, 7 and 15
// CSAs per step), plus one of 32 inputs.
constexpr int kMinLogd = 2;
static StreamKernel csa_table[3][4] = {
    {csa_kernel<8, 2>, csa_kernel<8, 3>, csa_kernel<8, 4>, csa_kernel<8, 5>},
    {csa_kernel<16, 2>, csa_kernel<16, 3>, csa_kernel<16, 4>, csa_kernel<16, 5>},
    {csa_kernel<32, 2>, csa_kernel<32, 3>, csa_kernel<32, 4>, csa_kernel<32, 5>},
};
static StreamKernel ballot_table[3] = {ballot_kernel<8>, ballot_kernel<16>, ballot_kernel<32>};
static StreamKernel hybrid_table[3][4] = {
    {hybrid_kernel<8, 2>, hybrid_kernel<8, 3>, hybrid_kernel<8, 4>, hybrid_kernel<8, 5>},
    {hybrid_kernel<16, 2>, hybrid_kernel<16, 3>, hybrid_kernel<16, 4>, hybrid_kernel<16, 5>},
    {hybrid_kernel<32, 2>, hybrid_kernel<32, 3>, hybrid_kernel<32, 4>, hybrid_kernel<32, 5>},
};
static CeilKernel ceil_table[4] = {ceiling_kernel<2>, ceiling_kernel<3>, ceiling_kernel<4>,
                                   ceiling_kernel<5>};

// Default launch shape per width and size, measured on MI355X over 256 MiB - 16 GiB
// inputs: a circuit of 16 dwords per lane per step (as many inputs as the paper's
// 1 kB circuit) and few waves -- 3 to 4 per compute unit, each with two 4 KiB tiles
// in flight, about 8 MiB in flight over the chip.  More resident waves lower the
// achieved bandwidth (6.9 TB/s at full occupancy against 7.2 TB/s).  Above 1 GiB,
// 8- and 32-bit words do best with three 64-thread blocks per CU; up to 1 GiB, and
// for 16-bit words at every size, one 256-thread block per CU (for 256 MiB of u32
// words 6.3 TB/s against 4.9).
struct Shape {
    int logd, threads, waves_per_cu;
};
static Shape default_shape(int k, uint64_t nbytes) {
    if (k == 16 || nbytes <= (1ull << 30)) return {4, 256, 4};
    return {4, 64, 3};
}
// The hybrid kernel issues 32 ballots and scalar adds per carry besides the
// circuit: six 64-thread blocks per CU (6.97-6.98 TB/s over 16 GiB at every
// width) against 5.4-6.0 TB/s at the counting kernel's shapes.
static Shape hybrid_shape() { return {4, 64, 6}; }
static int default_logd(int k) { return default_shape(k, 0).logd; }

// Resident blocks per CU of a kernel at a block size (cached).
static int occupancy(const void* kernel, int threads) {
    static std::mutex mu;
    static const void* keys[64];
    static int tvals[64], vals[64], used = 0;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
        if (keys[i] == kernel && tvals[i] == threads) return vals[i];
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess ||
        nb <= 0)
        nb = 2;
    if (used < 64) {
        keys[used] = kernel;
        tvals[used] = threads;
        vals[used] = nb;
        ++used;
    }
    return nb;
}

static const void* kernel_of(int variant, int k, int logd) {
    if (variant == PPC_VARIANT_BALLOT) return (const void*)ballot_table[class_index(k)];
    if (variant == PPC_VARIANT_HYBRID)
        return (const void*)hybrid_table[class_index(k)][logd - kMinLogd];
    return (const void*)csa_table[class_index(k)][logd - kMinLogd];
}

int resolve_launch(const ppc_launch_config* cfg, int k, uint64_t units, bool has_edges,
                   uint64_t nbytes, Launch* out) {
    ppc_launch_config c = {};
    if (cfg) c = *cfg;
    if (c.variant != PPC_VARIANT_CSA && c.variant != PPC_VARIANT_BALLOT &&
        c.variant != PPC_VARIANT_HYBRID)
        return PPC_ERR_ARG;
    int logd = default_logd(k);
    if (c.depth) {
        logd = logd_of_depth(c.depth);
        if (logd < 0) return PPC_ERR_ARG;
    }
    const Shape shape = c.variant == PPC_VARIANT_HYBRID ? hybrid_shape() : default_shape(k, nbytes);
    const int threads = c.block_threads ? c.block_threads : shape.threads;
    if (threads < kWave || threads > kMaxThreads || threads % kWave) return PPC_ERR_ARG;
    if (c.blocks_per_cu < 0 || c.grid < 0) return PPC_ERR_ARG;

    const DeviceFacts* dev = nullptr;
    int st = current_device(&dev);
    if (st) return st;
    const int wpb = threads / kWave;
    const uint64_t tile_units =
        c.variant == PPC_VARIANT_BALLOT ? (uint64_t)kWave : (uint64_t)kWave * ((1u << logd) / 4);
    const uint64_t tiles = (units + tile_units - 1) / tile_units;
    uint64_t need = blocks_needed(tiles, wpb);
    if (need == 0) need = has_edges ? 1 : 0;
    int64_t grid;
    if (c.grid > 0) {
        grid = c.grid;
    } else {
        int bpc = c.blocks_per_cu;
        if (!bpc) {
            // The counting kernels are memory bound and run best with few waves
            // (the hybrid with six per CU); the ballot kernel is ALU bound and
            // wants every wave that fits.
            if (c.variant == PPC_VARIANT_BALLOT)
                bpc = occupancy(kernel_of(c.variant, k, logd), threads);
            else
                bpc = (shape.waves_per_cu + wpb - 1) / wpb;
        }
        grid = (int64_t)bpc * dev->cus;
        if ((uint64_t)grid > need) grid = (int64_t)need;
    }
    // Keep every block's per-class total below 2^32: a class gathers at most one
    // bit per input byte, so no block may take 2^32 bytes or more.
    const int64_t min_grid = (int64_t)(nbytes >> 31) + 1;
    if (grid < min_grid) grid = min_grid;
    if (grid < 1) grid = 1;
    if (grid > 0x7fffffff) return PPC_ERR_ARG;
    out->variant = c.variant;
    out->logd = logd;
    out->threads = threads;
    out->grid = grid;
    return PPC_OK;
}

// The call's configuration with the environment's overrides in its zero fields.
static int merged_config(int k, const ppc_launch_config* cfg, ppc_launch_config* out) {
    *out = cfg ? *cfg : ppc_launch_config{};
    const EnvLaunch& e = env_launch(k);
    if (!e.set) return PPC_OK;
    if (e.bad) return PPC_ERR_ARG;
    if (!out->variant) out->variant = e.cfg.variant;
    if (!out->depth) out->depth = e.cfg.depth;
    if (!out->block_threads) out->block_threads = e.cfg.block_threads;
    if (!out->blocks_per_cu) out->blocks_per_cu = e.cfg.blocks_per_cu;
    if (!out->grid) out->grid = e.cfg.grid;
    return PPC_OK;
}

int launch_stream(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream,
                  const ppc_launch_config* cfg_in) {
    if (k != 8 && k != 16 && k != 32 && k != 64) return PPC_ERR_WIDTH;
    if (n == 0) return PPC_OK;
    ppc_launch_config merged;
    if (int mst = merged_config(k, cfg_in, &merged)) return mst;
    const ppc_launch_config* cfg = &merged;
    if (k == 64) return launch_wide64(ptr, n, counts, stream, cfg);
    uint64_t nbytes = 0;
    int st = check_stream_args(ptr, n, k, counts, &nbytes);
    if (st != PPC_OK || nbytes == 0) return st;
    const Split s = split_stream(ptr, nbytes, k);
    Launch L;
    st = resolve_launch(cfg, k, s.units, s.head_len + s.tail_len > 0, nbytes, &L);
    if (st) return st;
    Edges e{s.head, s.tail, s.head_len, s.tail_len};
    const u32x4* body = (const u32x4*)s.body;
    uint64_t units = s.units;
    uint32_t rot = s.rot;
    unsigned long long* cp = (unsigned long long*)counts;
    void* args[] = {&body, &units, &e, &k, &rot, &cp};
    const void* kern = kernel_of(L.variant, k, L.logd);
    PPC_HIP(hipLaunchKernel(kern, dim3((uint32_t)L.grid), dim3(L.threads), args, 0,
                            (hipStream_t)stream));
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

extern "C" {

int pospopcnt_u8(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream) {
    return launch_stream(ptr, n, 8, counts, stream, nullptr);
}
int pospopcnt_u16(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream) {
    return launch_stream(ptr, n, 16, counts, stream, nullptr);
}
int pospopcnt_u32(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream) {
    return launch_stream(ptr, n, 32, counts, stream, nullptr);
}
int pospopcnt(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream) {
    return launch_stream(ptr, n, k, counts, stream, nullptr);
}
int pospopcnt_ex(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream,
                 const ppc_launch_config* config) {
    return launch_stream(ptr, n, k, counts, stream, config);
}

int ppc_read_ceiling(const void* ptr, uint64_t nbytes, uint64_t* sink, ppc_stream stream,
                     const ppc_launch_config* config) {
    if (nbytes == 0) return PPC_OK;
    if (!ptr || !sink) return PPC_ERR_NULL;
    if ((uintptr_t)sink & 7u) return PPC_ERR_ALIGN;
    if ((uintptr_t)ptr + nbytes < (uintptr_t)ptr) return PPC_ERR_RANGE;
    const Split s = split_stream(ptr, nbytes, 8);
    ppc_launch_config c = {};
    if (config) c = *config;
    c.variant = PPC_VARIANT_CSA;
    Launch L;
    int st = resolve_launch(&c, 16, s.units, s.head_len + s.tail_len > 0, nbytes, &L);
    if (st) return st;
    Edges e{s.head, s.tail, s.head_len, s.tail_len};
    const u32x4* body = (const u32x4*)s.body;
    uint64_t units = s.units;
    unsigned long long* sp = (unsigned long long*)sink;
    void* args[] = {&body, &units, &e, &sp};
    PPC_HIP(hipLaunchKernel((const void*)ceil_table[L.logd - kMinLogd], dim3((uint32_t)L.grid),
                            dim3(L.threads), args, 0, (hipStream_t)stream));
    return PPC_OK;
}

}  // extern "C"
