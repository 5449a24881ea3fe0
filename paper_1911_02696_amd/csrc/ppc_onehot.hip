// ppc_onehot.hip -- histogram of categorical ids as the positional population
// count of their one-hot codes, without writing the codes anywhere.
//
// The paper's motivating use (Sec. 1, Table 1): with `bins` categories, category
// c is bit c of a bins-bit one-hot word, and the positional population count of
// the encoded stream is the frequency histogram.  Here each lane loads raw ids
// (u8 or u16) with the same nontemporal dwordx4 tiles as the counting kernel,
// turns them into packed one-hot codes of C = 8, 16 or 32 bits in registers (the
// narrowest width that holds bins; see Codes: four 8-bit, two 16-bit or one 32-bit
// code per dword; ids >= C have no code), and feeds the code dwords of a tile to
// one Harley-Seal circuit of Sec. 2, whose carry enters the cross-tile levels of
// ppc_tree.h before it is counted per category class as in the counting kernel.
// Every id with a code adds one to exactly one class, so the ids >= C are the ids
// a lane saw less the sum of its class totals; the classes bins .. C-1 join them
// at the flush.
// Head and tail ids outside the 16-byte aligned body are expanded one per lane by
// the first wave; padding never becomes an id.
#include "ppc_device.h"
#include "ppc_internal.h"
#include "ppc_tree.h"

namespace ppc {

constexpr int kOnehotThreads = 256;

// Packed one-hot codes.  A code needs only C bits, so a 32-bit "code dword" holds
// 32 / C codes (C = 8: four bytes, C = 16: two halves, C = 32: one dword) and the
// circuit's class masks (mask_of<C>) merge them: class i collects bit i of every
// code in the dword.  A tile is 16 input dwords per lane (four dwordx4 loads):
// 16 * (4 / IDB) ids, hence NCODE = 2 C / IDB code dwords, one circuit of that
// many inputs.
template <int C, int IDB>
struct Codes {
    static constexpr int IDS_PER_IN = 4 / IDB;
    static constexpr int CODES_PER_DW = 32 / C;
    static constexpr int NIN = 16;
    static constexpr int NCODE = NIN * IDS_PER_IN / CODES_PER_DW;
    static constexpr int LOGC = C == 8 ? 3 : C == 16 ? 4 : 5;
    static constexpr uint32_t LANE = IDB == 1 ? 0x01010101u : 0x00010001u;  // 1 per id lane
    static constexpr uint32_t IDMASK = IDB == 1 ? 0xFFu : 0xFFFFu;
    // Input bits that are zero in every input dword whose ids are all < C.
    static constexpr uint32_t BAD = LANE * (IDMASK & ~(uint32_t)(C - 1));


    // The masked path: a tile that may hold ids >= C, or dwords that are not
    // input (unit[i] false: the missing units of a partial tile).  Those ids must
    // add nothing to the classes; each gets a stand-in code that take_back() later
    // removes, *ph counting the stand-ins:
    // - C = 8 (make_masked): the byte table of make() applied to the raw ids (u8)
    //   or to their low bytes (u16).  Selectors 8..11 copy the sign of table
    //   bytes 1, 3, 5, 7 (0x02, 0x08, 0x20: zero; 0x80: 0xFF), 12 gives zero and
    //   13..255 give 0xFF, so a byte of the result is a one-hot code (one bit) or
    //   an id >= 8 (0x00, or 0xFF: one in every class).  A u16 id whose high byte
    //   is not zero is cleared by the mask table below applied to its high byte.
    //   Bits 0 and 1 both set mark exactly the 0xFF bytes; *ph counts them.
    // - C = 16, 32 (clear_ids, then make): every id >= C becomes id 0 in place,
    //   whose code lands in class 0.  For u8 ids a byte table gives a mask of all
    //   ones per such id (table {0xFFFFFFFF : 0xFFFFFF00}: 0x00 at index 0, 0xFF
    //   elsewhere), indexed by the id's bits above LOGC: bits 5..7 for C = 32; bits
    //   4..7 for C = 16, with bit 3 of the index also set in bit 0 so that selector
    //   12, which gives zero, never occurs and 8..11 copy the sign of a 0xFF byte;
    //   *ph adds the mask's popcount, 8 per such id.  For u16 ids one packed
    //   16-bit minimum clamps each id to C: an id < C keeps its value, which has
    //   bit LOGC clear, and an id >= C becomes C, which has only bit LOGC set, so
    //   that bit counts the stand-ins (*ph adds one per such id) and keeping the
    //   bits below LOGC turns them into id 0.
    static constexpr bool CLEARS_IDS = C != 8;

    __device__ static __forceinline__ void make_masked(uint32_t* code, const uint32_t* in,
                                                       const bool* unit, uint32_t* ph) {
        static_assert(!CLEARS_IDS, "C = 16, 32 go through clear_ids");
        if constexpr (C == 8 && IDB == 1) {
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
                const uint32_t raw = __builtin_amdgcn_perm(0x80402010u, 0x08040201u, in[i]);
                const uint32_t ff = raw & (raw >> 1) & 0x01010101u;
                code[i] = unit[i] ? raw : 0u;
                *ph += unit[i] ? (uint32_t)__builtin_popcount(ff) : 0u;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NIN / 2; ++i) {
                const uint32_t lo = in[2 * i], hi = in[2 * i + 1];
                // low and high bytes of the four ids
                const uint32_t lb = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
                const uint32_t hb = __builtin_amdgcn_perm(hi, lo, 0x07050301u);
                const uint32_t mh =
                    __builtin_amdgcn_perm(0xFFFFFFFFu, 0xFFFFFF00u, hb | ((hb >> 3) & 0x01010101u));
                const uint32_t c = __builtin_amdgcn_perm(0x80402010u, 0x08040201u, lb) & ~mh;
                const uint32_t ff = c & (c >> 1) & 0x01010101u;
                // both dwords of a pair lie in one 16-byte unit
                code[i] = unit[2 * i] ? c : 0u;
                *ph += unit[2 * i] ? (uint32_t)__builtin_popcount(ff) : 0u;
            }
        }
    }

    __device__ static __forceinline__ void clear_ids(uint32_t* in, const bool* unit,
                                                     uint32_t* ph) {
        if constexpr (IDB == 2) {
            typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
            const u16x2 cc = {(unsigned short)C, (unsigned short)C};
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
                uint32_t cl = __builtin_bit_cast(
                    uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, in[i]), cc));
                cl = unit[i] ? cl : LANE * C;  // a missing unit: two stand-ins
                *ph += (uint32_t)__builtin_popcount(cl & (LANE * C));
                in[i] = cl & (LANE * (C - 1));
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            uint32_t m;
            if constexpr (C == 32) {
                m = __builtin_amdgcn_perm(0xFFFFFFFFu, 0xFFFFFF00u, (in[i] >> 5) & 0x07070707u);
            } else {
                const uint32_t h = (in[i] >> 4) & 0x0F0F0F0Fu;
                m = __builtin_amdgcn_perm(0xFFFFFFFFu, 0xFFFFFF00u, h | ((h >> 3) & 0x01010101u));
            }
            m = unit[i] ? m : 0xFFFFFFFFu;
            *ph += (uint32_t)__builtin_popcount(m);
            in[i] &= ~m;
        }
    }

    // Removes from a lane's class totals what the stand-in codes added.
    __device__ static __forceinline__ void take_back(uint32_t (&tot)[C], uint32_t ph) {
        if constexpr (C == 8) {
#pragma unroll
            for (int i = 0; i < C; ++i) tot[i] -= ph;
        } else if constexpr (IDB == 2) {
            tot[0] -= ph;  // one per stand-in id
        } else {
            tot[0] -= ph / 8;  // eight mask bits per stand-in id
        }
    }

    // Code dwords of NIN input dwords whose ids are all below C.  C = 8: one
    // byte-table lookup per four codes (v_perm_b32: byte b of the result is byte
    // sel_b of {S0:S1}; the table {0x80402010 : 0x08040201} holds 1 << j at byte
    // j).  C = 16: packed 16-bit shifts, two codes per op.  C = 32: one byte- or
    // word-selecting shift per id.
    __device__ static __forceinline__ void make(uint32_t* code, const uint32_t* in) {
        if constexpr (C == 8) {
            if constexpr (IDB == 1) {
#pragma unroll
                for (int i = 0; i < NIN; ++i)
                    code[i] = __builtin_amdgcn_perm(0x80402010u, 0x08040201u, in[i]);
            } else {
#pragma unroll
                for (int i = 0; i < NIN / 2; ++i) {
                    // the four id bytes, then the table lookup
                    const uint32_t sel = __builtin_amdgcn_perm(in[2 * i + 1], in[2 * i], 0x06040200u);
                    code[i] = __builtin_amdgcn_perm(0x80402010u, 0x08040201u, sel);
                }
            }
        } else if constexpr (C == 16) {
            typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
            const u16x2 one = {1, 1};
            if constexpr (IDB == 1) {
#pragma unroll
                for (int i = 0; i < NIN; ++i) {
                    // ids 0 and 1 (2 and 3) widened to the two 16-bit shift amounts
                    const uint32_t a = __builtin_amdgcn_perm(0u, in[i], 0x0C010C00u);
                    const uint32_t b = __builtin_amdgcn_perm(0u, in[i], 0x0C030C02u);
                    code[2 * i] = __builtin_bit_cast(uint32_t, one << __builtin_bit_cast(u16x2, a));
                    code[2 * i + 1] =
                        __builtin_bit_cast(uint32_t, one << __builtin_bit_cast(u16x2, b));
                }
            } else {
#pragma unroll
                for (int i = 0; i < NIN; ++i)
                    code[i] = __builtin_bit_cast(uint32_t, one << __builtin_bit_cast(u16x2, in[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
#pragma unroll
                for (int j = 0; j < IDS_PER_IN; ++j) {
                    const int sh = 32 / IDS_PER_IN * j;
                    code[i * IDS_PER_IN + j] = 1u << ((in[i] >> sh) & IDMASK);
                }
            }
        }
    }
};

template <int C, int IDB, int LOGD>
__device__ __forceinline__ uint32_t onehot_step(uint32_t (&B)[LOGD], uint32_t& ph,
                                                const u32x4 (&v)[4], const bool (&valid)[4],
                                                bool maybe_partial) {
    using K = Codes<C, IDB>;
    static_assert(K::NCODE == (1 << LOGD), "one circuit per tile");
    uint32_t in[K::NIN];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        in[4 * j + 0] = v[j].x;
        in[4 * j + 1] = v[j].y;
        in[4 * j + 2] = v[j].z;
        in[4 * j + 3] = v[j].w;
    }
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < K::NIN; ++i) any |= in[i];
    const uint32_t bad = any & K::BAD;
    uint32_t code[K::NCODE];
    // Wave-uniform choice: ids are masked only when some lane holds an id >= C or
    // the tile is the partial last one (whose missing units carry no ids at all).
    const bool clean = !maybe_partial && __ballot(bad != 0) == 0;
    bool unit[K::NIN];
#pragma unroll
    for (int i = 0; i < K::NIN; ++i) unit[i] = valid[i / 4];
    // Each branch runs its own copy of the circuit, so that no code or id is live
    // across the join (a value merged there costs a register copy per id on the
    // fast path).
    if (clean) {
        K::make(code, in);
        return Circuit<LOGD>::run(B, code);
    }
    if constexpr (K::CLEARS_IDS) {
        // The same codes as the fast path once the ids are cleared, fed to the
        // circuit in reverse order so that the compiler does not merge the two
        // branches' code: the circuit keeps every class's weighted sum whatever
        // the order of its inputs.
        K::clear_ids(in, unit, &ph);
        K::make(code, in);
        uint32_t rev[K::NCODE];
#pragma unroll
        for (int i = 0; i < K::NCODE; ++i) rev[i] = code[K::NCODE - 1 - i];
        return Circuit<LOGD>::run(B, rev);
    } else {
        K::make_masked(code, in, unit, &ph);
        return Circuit<LOGD>::run(B, code);
    }
}

// The id at head or tail position `lane` of the first wave: lanes 0..15 take
// head ids, lanes 16..31 tail ids.  u16 ids are 2-byte aligned, so the head and
// tail hold whole ids.  `seen` counts the id.
template <int C, int IDB>
__device__ __forceinline__ uint32_t edge_onehot(const Edges& e, int lane, uint32_t& seen) {
    const uint8_t* p = nullptr;
    if (lane < 16) {
        if ((uint32_t)(lane * IDB) < e.head_len) p = e.head + lane * IDB;
    } else if (lane < 32) {
        if ((uint32_t)((lane - 16) * IDB) < e.tail_len) p = e.tail + (lane - 16) * IDB;
    }
    if (!p) return 0u;
    const uint32_t id = IDB == 1 ? (uint32_t)p[0] : (uint32_t)p[0] | ((uint32_t)p[1] << 8);
    ++seen;
    return id < (uint32_t)C ? 1u << id : 0u;
}

// Tiles in flight per wave while one is turned into codes and counted: three for u8
// ids, whose tiles cost the most VALU per byte (a wave's next two tiles load while it
// works through one), two for u16 ids.  Measured over 16 GiB of ids per launch at the
// default shapes: u8 ids with 32 categories 7208-7210 GB/s against 6859-6862 with two;
// with 8 categories and 1% of the ids outside them 7325 against 6921-6935; u16 ids ran
// 1-2.5% slower with three.
constexpr int onehot_inflight(int code_bits, int id_bytes) {
    return (void)code_bits, id_bytes == 1 ? 3 : 2;
}

// bins <= C categories counted with C-bit codes: classes bins .. C-1 hold ids that
// have a code but no category, and are flushed into counts[bins] with the rest.
template <int C, int IDB>
__global__ void __launch_bounds__(kOnehotThreads)
onehot_kernel(const u32x4* __restrict__ body, uint64_t units, Edges edges, uint32_t bins,
              unsigned long long* __restrict__ counts) {
    constexpr int U = 4;
    constexpr int LOGD = C == 8 ? (IDB == 1 ? 4 : 3) : C == 16 ? (IDB == 1 ? 5 : 4)
                                                                : (IDB == 1 ? 6 : 5);
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wave;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t full = units / TILE;

    // Levels past the tile: more for wider codes, whose per-class count costs more.
    constexpr int E = C == 8 ? 1 : C == 16 ? 2 : 3;
    // ph: stand-in codes of the masked path (Codes::make_masked)
    uint32_t B[LOGD], ph = 0;
#pragma unroll
    for (int j = 0; j < LOGD; ++j) B[j] = 0;
    TileTree<C, LOGD, E> tree;
    tree.init();
    const bool all[U] = {true, true, true, true};
    walk_tiles_p<U, onehot_inflight(C, IDB)>(body, full, gw, nw, lane, [&](const u32x4(&v)[U]) {
        tree.add(onehot_step<C, IDB, LOGD>(B, ph, v, all, false));
    });
    // ids this lane has seen: 4 / IDB per input dword, 16 dwords per tile
    uint32_t seen = tree.tiles * (16u * 4u / IDB);
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 t[U];
        load_tile_masked<U>(t, body + full * TILE + lane, lane, rem);
        bool valid[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            valid[j] = (uint64_t)(j * kWave + lane) < rem;
            seen += valid[j] ? 4u * 4u / IDB : 0u;
        }
        tree.add(onehot_step<C, IDB, LOGD>(B, ph, t, valid, true));
    }
    const uint32_t e = (blockIdx.x == 0 && wave == 0) ? edge_onehot<C, IDB>(edges, lane, seen) : 0u;

    uint32_t tot[C], other = seen;
    tree.totals(tot, B, e);
    Codes<C, IDB>::take_back(tot, ph);
#pragma unroll
    for (int i = 0; i < C; ++i) other -= tot[i];
    const uint32_t v = wave_reduce_scatter<C>(tot, lane);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) other += (uint32_t)__shfl_xor((int)other, o, kWave);
    __shared__ uint32_t red[kOnehotThreads / kWave][C];
    __shared__ uint32_t red_other[kOnehotThreads / kWave];
    constexpr int G = kWave / C;
    if (lane % G == 0) red[wave][lane / G] = v;
    if (lane == 0) red_other[wave] = other;
    __syncthreads();
    const uint32_t p = threadIdx.x;
    if (p < bins) {
        unsigned long long s = 0;
        for (int w = 0; w < wpb; ++w) s += red[w][p];
        if (s) atomicAdd(counts + p, s);
    } else if (p == bins) {
        unsigned long long s = 0;
        for (int w = 0; w < wpb; ++w) {
            s += red_other[w];
            for (int cls = (int)bins; cls < C; ++cls) s += red[w][cls];
        }
        if (s) atomicAdd(counts + bins, s);
    }
}

using OnehotKernel = void (*)(const u32x4*, uint64_t, Edges, uint32_t, unsigned long long*);

static const void* onehot_of(int code_bits, int id_bytes) {
    static OnehotKernel table[2][3] = {
        {onehot_kernel<8, 1>, onehot_kernel<16, 1>, onehot_kernel<32, 1>},
        {onehot_kernel<8, 2>, onehot_kernel<16, 2>, onehot_kernel<32, 2>},
    };
    return (const void*)table[id_bytes - 1][code_bits == 8 ? 0 : code_bits == 16 ? 1 : 2];
}

// Default launch shape per (categories, id width), from a sweep of block sizes 64..256
// and 1..12 blocks per CU over 16 GiB of ids on MI355X.  Few waves win, as for the
// counting kernel: three per CU for 8 categories, whose codes cost one op per four
// u8 ids, and four (one per SIMD) where a tile costs more arithmetic (16 or 32
// categories, or ids outside the categories, which take the masked path).
struct OnehotShape {
    int threads, blocks_per_cu;
};

static OnehotShape onehot_shape(int code_bits) {
    return code_bits == 8 ? OnehotShape{64, 3} : OnehotShape{256, 1};
}

static int launch_histogram(const void* ids, uint64_t n, int id_bytes, int bins,
                            uint64_t* counts, ppc_stream stream, const ppc_launch_config* cfg) {
    if (id_bytes != 1 && id_bytes != 2) return PPC_ERR_ARG;
    if (bins < 1 || bins > 32) return PPC_ERR_WIDTH;
    // codes of 8, 16 or 32 bits: the narrowest that holds every category
    const int code_bits = bins <= 8 ? 8 : bins <= 16 ? 16 : 32;
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
    const OnehotShape dflt = onehot_shape(code_bits);
    const int threads = c.block_threads ? c.block_threads : dflt.threads;
    if (threads < kWave || threads > kOnehotThreads || threads % kWave) return PPC_ERR_ARG;
    if (c.blocks_per_cu < 0 || c.grid < 0) return PPC_ERR_ARG;
    const DeviceFacts* dev = nullptr;
    int st = current_device(&dev);
    if (st) return st;
    const Split s = split_stream(ids, nbytes, 8);
    const int wpb = threads / kWave;
    const uint64_t tiles = (s.units + kWave * 4 - 1) / (kWave * 4);
    uint64_t need = blocks_needed(tiles, wpb);
    if (need == 0) need = 1;
    int64_t grid;
    if (c.grid > 0) {
        grid = c.grid;
    } else {
        const int bpc = c.blocks_per_cu ? c.blocks_per_cu : dflt.blocks_per_cu;
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
    uint32_t nbins = (uint32_t)bins;
    void* args[] = {&body, &units, &e, &nbins, &cp};
    PPC_HIP(hipLaunchKernel(onehot_of(code_bits, id_bytes), dim3((uint32_t)grid), dim3(threads), args,
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
