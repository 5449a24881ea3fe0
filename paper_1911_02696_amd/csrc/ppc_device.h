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

// Reduce-scatter of C per-lane values over a wave: each exchange at distance
// o = 32, 16, ... halves the values a lane keeps (the lower lane of a pair keeps
// the lower half of the classes, the upper lane the upper half), then the last
// exchanges are plain butterflies.  Afterwards every lane holds the wave total
// of class  lane / (64 / C).  C - 1 + log2(64 / C) exchanges instead of 6 C.
template <int C>
__device__ __forceinline__ uint32_t wave_reduce_scatter(uint32_t (&v)[C], int lane) {
    int width = C;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        if (width > 1) {
            const bool upper = (lane & o) != 0;
#pragma unroll
            for (int j = 0; j < C / 2; ++j) {
                if (j < width / 2) {
                    const uint32_t send = upper ? v[j] : v[j + width / 2];
                    const uint32_t keep = upper ? v[j + width / 2] : v[j];
                    v[j] = keep + (uint32_t)__shfl_xor((int)send, o, kWave);
                }
            }
            width >>= 1;
        } else {
            v[0] += (uint32_t)__shfl_xor((int)v[0], o, kWave);
        }
    }
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

}  // namespace ppc
