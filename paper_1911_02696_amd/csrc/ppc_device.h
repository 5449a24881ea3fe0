// ppc_device.h -- device building blocks of the gfx950 positional popcount.
//
// Layout convention.  The kernels read the input as 32-bit little-endian dwords
// (16-byte dwordx4 loads).  Bit i of a dword belongs to a "class" of dword bit
// positions that all map to the same word bit:
//   C = 8  classes (k = 8):  class i = dword bits {i, i+8, i+16, i+24}
//   C = 16 classes (k = 16): class i = dword bits {i, i+16}
//   C = 32 classes (k = 32): class i = dword bit  {i}
// A class is counted with one AND + one population count (mask_of<C>(i)).
// When the stream starts at byte address ptr with r = ptr mod (k/8), dword bit
// i holds word bit (i - 8r) mod k, so class i is added to counts[(i - 8r) mod k]
// at the flush; this one rotation handles every start alignment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ppc {

constexpr int kWave = 64;

// Four dwords, as one 16-byte load.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Carry-save adder (Sec. 2): l = a xor b xor c, h = majority(a, b, c).  gfx950's
// three-input bitwise op takes the truth table as an 8-bit immediate, the same
// encoding Sec. 3 derives for the AVX-512 ternary-logic instruction (Table 2:
// 0x96 for the sum bit, 0xE8 for the carry bit), so one CSA is two VALU ops.
__device__ __forceinline__ void csa(uint32_t& h, uint32_t& l, uint32_t a, uint32_t b,
                                    uint32_t c) {
    h = __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
    l = __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Harley-Seal circuit over 2^N dwords (Sec. 2): F_1 is one CSA of the running
// plane B[0] with two inputs; F_N runs F_{N-1} on each half of its inputs, the
// second call continuing from the planes the first left, and combines the plane
// B[N-1] it was given with the two weight-2^(N-1) carries of the halves in one
// more CSA.  Updates B[0 .. N-1] (weights 1 .. 2^(N-1)) and returns the carry of
// weight 2^N.  2^N - 1 CSAs in all.
template <int N>
struct Circuit {
    __device__ __forceinline__ static uint32_t run(uint32_t* B, const uint32_t* d) {
        const uint32_t x = Circuit<N - 1>::run(B, d);
        const uint32_t y = Circuit<N - 1>::run(B, d + (1 << (N - 1)));
        uint32_t h, l;
        csa(h, l, B[N - 1], x, y);
        B[N - 1] = l;
        return h;
    }
};
template <>
struct Circuit<1> {
    __device__ __forceinline__ static uint32_t run(uint32_t* B, const uint32_t* d) {
        uint32_t h, l;
        csa(h, l, B[0], d[0], d[1]);
        B[0] = l;
        return h;
    }
};

template <int C>
__device__ __forceinline__ constexpr uint32_t mask_of(int i) {
    return C == 8 ? (0x01010101u << i) : C == 16 ? (0x00010001u << i) : (1u << i);
}

// cnt[i] += number of set bits of x in class i (AND + popcount-accumulate, the
// per-position counting of the carry register of Sec. 4.1 / Fig. 6).
template <int C>
__device__ __forceinline__ void count_classes(uint32_t (&cnt)[C], uint32_t x) {
#pragma unroll
    for (int i = 0; i < C; ++i) cnt[i] = __builtin_popcount(x & mask_of<C>(i)) + cnt[i];
}

// Per-lane totals: carry counts carry the deferred weight 2^LOGD; the running
// planes B[j] are flushed with weights 2^j (Sec. 4.1); e is a partial dword
// counted with weight 1.
template <int C, int LOGD>
__device__ __forceinline__ void lane_totals(uint32_t (&out)[C], const uint32_t (&cnt)[C],
                                            const uint32_t (&B)[LOGD], uint32_t e) {
#pragma unroll
    for (int i = 0; i < C; ++i) {
        uint32_t t = (cnt[i] << LOGD) + __builtin_popcount(e & mask_of<C>(i));
#pragma unroll
        for (int j = 0; j < LOGD; ++j) t += __builtin_popcount(B[j] & mask_of<C>(i)) << j;
        out[i] = t;
    }
}

// Bit-sliced ("vertical") counter of carry planes: plane V[j] holds bit j of the
// number of carries seen so far at each dword bit position, so a carry plane is
// added with a ripple of half adders (2 ops per plane) whatever the number of
// classes.  It is the Sec. 2 idea of keeping a sum as bit planes, carried past
// the circuit's own planes; with L planes it holds up to 2^L - 1 carries.
template <int L>
__device__ __forceinline__ void vertical_add(uint32_t (&V)[L], uint32_t c) {
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t t = V[j] & c;
        V[j] ^= c;
        c = t;
    }
}

// out[i] += per-lane class-i total of planes P[0..L) with weights 2^(shift + j).
template <int C, int L>
__device__ __forceinline__ void add_plane_totals(uint32_t (&out)[C], const uint32_t (&P)[L],
                                                 int shift) {
#pragma unroll
    for (int i = 0; i < C; ++i) {
        uint32_t t = 0;
#pragma unroll
        for (int j = 0; j < L; ++j) t += __builtin_popcount(P[j] & mask_of<C>(i)) << j;
        out[i] += t << shift;
    }
}

// One exchange level at distance O of the reduce-scatter below, W values per lane
// still distinct: with W > 1 the lower lane of each pair keeps (and sums) the lower
// half of the values, the upper lane the upper half; with W = 1 it is a plain
// butterfly.  W and O are template arguments so that every index is a constant
// and the values stay in registers.
template <int W, int O>
__device__ __forceinline__ void reduce_scatter_levels(uint32_t* v, int lane) {
    if constexpr (O >= 1) {
        if constexpr (W > 1) {
            const bool upper = (lane & O) != 0;
#pragma unroll
            for (int j = 0; j < W / 2; ++j) {
                const uint32_t send = upper ? v[j] : v[j + W / 2];
                const uint32_t keep = upper ? v[j + W / 2] : v[j];
                v[j] = keep + (uint32_t)__shfl_xor((int)send, O, kWave);
            }
            reduce_scatter_levels<W / 2, O / 2>(v, lane);
        } else {
            v[0] += (uint32_t)__shfl_xor((int)v[0], O, kWave);
            reduce_scatter_levels<1, O / 2>(v, lane);
        }
    }
}

// Reduce-scatter of C per-lane values over a wave: each exchange at distance
// o = 32, 16, ... halves the values a lane keeps (the lower lane of a pair keeps
// the lower half of the classes, the upper lane the upper half), then the last
// exchanges are plain butterflies.  Afterwards every lane holds the wave total
// of class  lane / (64 / C).
// The two widest levels use gfx950's lane-swap instructions: swapping the upper
// 32 lanes of v[j] with the lower 32 lanes of v[j + h] leaves each lane holding
// both operands of its own sum, so a pair costs one swap and one add, in
// registers, with no select.  The narrow levels that follow use shuffles.
template <int C>
__device__ __forceinline__ uint32_t wave_reduce_scatter(uint32_t (&v)[C], int lane) {
    static_assert(C >= 4 && C <= 64, "class count");
#pragma unroll
    for (int j = 0; j < C / 2; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(v[j], v[j + C / 2], false, false);
        v[j] = r[0] + r[1];
    }
#pragma unroll
    for (int j = 0; j < C / 4; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(v[j], v[j + C / 4], false, false);
        v[j] = r[0] + r[1];
    }
    reduce_scatter_levels<C / 4, 8>(v, lane);
    return v[0];
}

// Sum the per-wave class totals of a block (red: [waves][C] in LDS, already
// filled) and add class i into counts[(i - rot) mod k] with one 64-bit
// device-scope atomic per nonzero word position.  C >= k; for C > k the classes
// that land on the same position are summed first.  Called by every thread of
// the block after a barrier.
template <int C>
__device__ __forceinline__ void block_flush(const uint32_t (*red)[C], int waves, int k,
                                            uint32_t rot, unsigned long long* counts) {
    const int p = threadIdx.x;
    if (p < k) {
        unsigned long long s = 0;
        for (int cls = (p + (int)rot) & (k - 1); cls < C; cls += k)
            for (int w = 0; w < waves; ++w) s += red[w][cls];
        if (s) atomicAdd(counts + p, s);
    }
}

// As block_flush, from 64-bit per-wave class totals.
template <int C>
__device__ __forceinline__ void block_flush64(const unsigned long long (*acc)[C], int waves,
                                              int k, uint32_t rot, unsigned long long* counts) {
    const int p = threadIdx.x;
    if (p < k) {
        unsigned long long s = 0;
        for (int cls = (p + (int)rot) & (k - 1); cls < C; cls += k)
            for (int w = 0; w < waves; ++w) s += acc[w][cls];
        if (s) atomicAdd(counts + p, s);
    }
}

// ---------------------------------------------------------------- stream walking

// Head and tail bytes of a stream (the parts outside its 16-byte aligned body).
struct Edges {
    const uint8_t* head;
    const uint8_t* tail;
    uint32_t head_len;
    uint32_t tail_len;
};

// Lanes 0..14 take one head byte each, lanes 16..30 one tail byte each; the byte
// is placed at its position inside its aligned dword.  Other lanes return 0.
__device__ __forceinline__ uint32_t edge_dword(const Edges& e, int lane) {
    const uint8_t* p = nullptr;
    if (lane < 16) {
        if ((uint32_t)lane < e.head_len) p = e.head + lane;
    } else if (lane < 32) {
        if ((uint32_t)(lane - 16) < e.tail_len) p = e.tail + (lane - 16);
    }
    if (!p) return 0u;
    return (uint32_t)(*p) << (8u * (uint32_t)((uintptr_t)p & 3u));
}

// Streaming loads carry the nontemporal hint: every byte is read exactly once, and
// on MI355X the hinted loads sustain about 15 % more HBM bandwidth than plain ones
// (7.1-7.2 TB/s against 6.2-6.3 TB/s for a read-only pass over 16 GiB).
// Input pointers are global memory; saying so keeps the loads global (not flat)
// also when the pointer was itself read from memory, as in the batched kernel.
typedef __attribute__((address_space(1))) const u32x4 global_u32x4;

__device__ __forceinline__ u32x4 stream_load(const u32x4* p) {
    return __builtin_nontemporal_load((global_u32x4*)p);
}

template <int U>
__device__ __forceinline__ void load_tile(u32x4 (&v)[U], const u32x4* __restrict__ p) {
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = stream_load(p + j * kWave);
}

// Masked load of the last, partial tile: loads past `rem` units read nothing and
// contribute zero dwords, which the circuit adds as nothing.
template <int U>
__device__ __forceinline__ void load_tile_masked(u32x4 (&v)[U], const u32x4* __restrict__ p,
                                                 int lane, uint64_t rem) {
#pragma unroll
    for (int j = 0; j < U; ++j)
        v[j] = ((uint64_t)(j * kWave + lane) < rem) ? stream_load(p + j * kWave)
                                                     : u32x4{0u, 0u, 0u, 0u};
}

// A tile consumer takes the loaded tile, and also the lane's address of it when
// it accepts a second argument (the copying consumers store the tile elsewhere).
template <int U, typename F>
__device__ __forceinline__ void consume_tile(F& consume, const u32x4 (&v)[U],
                                             const u32x4* p) {
    if constexpr (std::is_invocable_v<F&, const u32x4(&)[U], const u32x4*>)
        consume(v, p);
    else
        consume(v);
}

// Consume `count` whole tiles starting at p (already offset by the lane), each
// `stride` units after the previous, with two tiles in flight: the next tile's
// loads are issued before the current tile is consumed.  The trip count is known
// on entry and the loop body issues its loads without a condition, so the
// compiler's wait counters let the newer loads stay in flight while the older
// ones are consumed.
template <int U, typename F>
__device__ __forceinline__ void walk_n(const u32x4* __restrict__ p, uint64_t count,
                                       uint64_t stride, F&& consume) {
    if (count == 0) return;
    u32x4 a[U], b[U];
    load_tile<U>(a, p);
    while (count >= 3) {
        load_tile<U>(b, p + stride);
        consume_tile<U>(consume, a, p);
        load_tile<U>(a, p + 2 * stride);
        consume_tile<U>(consume, b, p + stride);
        p += 2 * stride;
        count -= 2;
    }
    if (count == 2) {
        load_tile<U>(b, p + stride);
        consume_tile<U>(consume, a, p);
        consume_tile<U>(consume, b, p + stride);
    } else {
        consume_tile<U>(consume, a, p);
    }
}

// ---------------------------------------------------------------- copying walks
//
// A copying count also writes every byte it reads to a destination that starts
// at the same address modulo 16 as the source, so that each 16-byte body unit of
// the source lands on one aligned 16-byte unit of the destination: delta =
// dst - src is a multiple of 16.  Stores are plain (cached): measured in the
// serving loop at 50,000 requests/s, they give lower latency than nontemporal
// stores (p50 / p99 0.034 / 0.148 ms against 0.036 / 0.172 ms), which sustain
// about 4% more requests/s at saturation.
typedef __attribute__((address_space(1))) u32x4 global_u32x4_w;

template <int U>
__device__ __forceinline__ void store_tile(const u32x4 (&v)[U], const u32x4* src_lane,
                                           intptr_t delta) {
    u32x4* q = (u32x4*)((const char*)src_lane + delta);
#pragma unroll
    for (int j = 0; j < U; ++j) *(global_u32x4_w*)(q + j * kWave) = v[j];
}

// Stores of the masked last tile: only the units below `rem`.
template <int U>
__device__ __forceinline__ void store_tile_masked(const u32x4 (&v)[U], const u32x4* src_lane,
                                                  intptr_t delta, int lane, uint64_t rem) {
    u32x4* q = (u32x4*)((const char*)src_lane + delta);
#pragma unroll
    for (int j = 0; j < U; ++j)
        if ((uint64_t)(j * kWave + lane) < rem) *(global_u32x4_w*)(q + j * kWave) = v[j];
}

// edge_dword, also writing the lane's edge byte (if any) to its place at delta.
__device__ __forceinline__ uint32_t edge_dword_copy(const Edges& e, int lane, intptr_t delta) {
    const uint8_t* p = nullptr;
    if (lane < 16) {
        if ((uint32_t)lane < e.head_len) p = e.head + lane;
    } else if (lane < 32) {
        if ((uint32_t)(lane - 16) < e.tail_len) p = e.tail + (lane - 16);
    }
    if (!p) return 0u;
    const uint8_t byte = *p;
    *(uint8_t*)(p + delta) = byte;
    return (uint32_t)byte << (8u * (uint32_t)((uintptr_t)p & 3u));
}

// As walk_n with P tiles in flight (P >= 2): P - 1 tiles are loaded ahead of the
// one being consumed.  The steady-state body handles P tiles with the buffer
// indices fixed at compile time; the last tiles (fewer than 2P - 1) are handled by
// an unrolled tail whose conditions are uniform over the wave.
template <int U, int P, typename F>
__device__ __forceinline__ void walk_np(const u32x4* __restrict__ p, uint64_t count,
                                        uint64_t stride, F&& consume) {
    static_assert(P >= 2, "at least two tiles in flight");
    if constexpr (P == 2) {
        walk_n<U>(p, count, stride, consume);
    } else {
        if (count == 0) return;
        u32x4 buf[P][U];
#pragma unroll
        for (int j = 0; j < P - 1; ++j)
            if ((uint64_t)j < count) load_tile<U>(buf[j], p + j * stride);
        while (count >= 2 * P - 1) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                load_tile<U>(buf[(j + P - 1) % P], p + (j + P - 1) * stride);
                consume_tile<U>(consume, buf[j], p + j * stride);
            }
            p += P * stride;
            count -= P;
        }
#pragma unroll
        for (int j = 0; j < 2 * P - 2; ++j) {
            if ((uint64_t)j < count) {
                if ((uint64_t)(j + P - 1) < count)
                    load_tile<U>(buf[(j + P - 1) % P], p + (j + P - 1) * stride);
                consume_tile<U>(consume, buf[j % P], p + j * stride);
            }
        }
    }
}

// Walk this wave's whole tiles t = gw, gw + nw, ... < full of a body.
template <int U, typename F>
__device__ __forceinline__ void walk_tiles(const u32x4* __restrict__ body, uint64_t full,
                                           uint64_t gw, uint64_t nw, int lane, F&& consume) {
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    if (gw >= full) return;
    walk_n<U>(body + gw * TILE + lane, (full - gw + nw - 1) / nw, nw * TILE, consume);
}

// As walk_tiles with P tiles in flight per wave.
template <int U, int P, typename F>
__device__ __forceinline__ void walk_tiles_p(const u32x4* __restrict__ body, uint64_t full,
                                             uint64_t gw, uint64_t nw, int lane, F&& consume) {
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    if (gw >= full) return;
    walk_np<U, P>(body + gw * TILE + lane, (full - gw + nw - 1) / nw, nw * TILE, consume);
}

template <int C, int LOGD, int U>
__device__ __forceinline__ void csa_step(uint32_t (&B)[LOGD], uint32_t (&cnt)[C],
                                         const u32x4 (&v)[U]) {
    static_assert(4 * U == (1 << LOGD), "one circuit per tile");
    uint32_t d[4 * U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        d[4 * j + 0] = v[j].x;
        d[4 * j + 1] = v[j].y;
        d[4 * j + 2] = v[j].z;
        d[4 * j + 3] = v[j].w;
    }
    count_classes<C>(cnt, Circuit<LOGD>::run(B, d));
}

// One stream's count, as block `block` of `blocks` working on it: the block's
// waves take whole tiles grid-stride (Sec. 4.1 per lane, two tiles in flight),
// the wave owning the last partial tile loads it masked, the first wave of block
// 0 adds the head and tail dwords, and the block adds its class totals into
// counts with rotation rot (see block_flush).  red is the block's LDS of
// [waves][C] class totals.  Called by every thread of the block.
template <int C, int LOGD>
__device__ __forceinline__ void count_stream(const u32x4* __restrict__ body, uint64_t units,
                                             const Edges& edges, int k, uint32_t rot,
                                             unsigned long long* __restrict__ counts,
                                             uint64_t block, uint64_t blocks,
                                             uint32_t (*red)[C]) {
    constexpr int U = (1 << LOGD) / 4;
    constexpr uint64_t TILE = (uint64_t)kWave * U;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const uint64_t gw = block * wpb + wave;
    const uint64_t nw = blocks * wpb;
    const uint64_t full = units / TILE;

    uint32_t B[LOGD];
    uint32_t cnt[C];
#pragma unroll
    for (int j = 0; j < LOGD; ++j) B[j] = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) cnt[i] = 0;

    walk_tiles<U>(body, full, gw, nw, lane,
                  [&](const u32x4(&v)[U]) { csa_step<C, LOGD, U>(B, cnt, v); });
    const uint64_t rem = units - full * TILE;
    if (rem != 0 && gw == full % nw) {
        u32x4 a[U];
        load_tile_masked<U>(a, body + full * TILE + lane, lane, rem);
        csa_step<C, LOGD, U>(B, cnt, a);
    }

    const uint32_t e = (block == 0 && wave == 0) ? edge_dword(edges, lane) : 0u;
    uint32_t tot[C];
    lane_totals<C, LOGD>(tot, cnt, B, e);
    const uint32_t v = wave_reduce_scatter<C>(tot, lane);
    constexpr int G = kWave / C;
    if (lane % G == 0) red[wave][lane / G] = v;
    __syncthreads();
    block_flush<C>(red, wpb, k, rot, counts);
}

}  // namespace ppc
