// ppc_tree.h -- the Harley-Seal recursion carried on past one tile's circuit.
#pragma once

#include "ppc_device.h"

namespace ppc {

// The Harley-Seal recursion of Sec. 2 carried on past the tile: F_{N+1} is two F_N
// and one CSA, so the carries of successive tile circuits (weight 2^LOGD each)
// enter E more levels.  Level e keeps a running plane R[e] and one pending carry
// P[e] of weight 2^(LOGD + e); the second carry to reach a level is merged with
// the pending one and R[e] by a CSA whose carry moves up a level.  Only carries
// leaving the top level are counted per class (Sec. 4.1), once every 2^E tiles.
// The tile number is the same in every lane, so the level choice is a scalar
// branch.
template <int C, int LOGD, int E>
struct TileTree {
    uint32_t R[E], P[E], cnt[C];
    uint32_t tiles;

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int e = 0; e < E; ++e) R[e] = P[e] = 0;
#pragma unroll
        for (int i = 0; i < C; ++i) cnt[i] = 0;
        tiles = 0;
    }

    __device__ __forceinline__ void add(uint32_t c) {
        bool up = true;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (up) {
                if (((tiles >> e) & 1u) == 0) {
                    P[e] = c;
                    up = false;
                } else {
                    uint32_t h, l;
                    csa(h, l, R[e], P[e], c);
                    R[e] = l;
                    P[e] = 0;
                    c = h;
                }
            }
        }
        if (up) count_classes<C>(cnt, c);
        ++tiles;
    }

    // Per-lane class totals: counted carries have weight 2^(LOGD + E), level e's
    // planes 2^(LOGD + e), the tile circuit's running planes B[j] 2^j; e0 is a
    // dword counted with weight 1.
    __device__ __forceinline__ void totals(uint32_t (&out)[C], const uint32_t (&B)[LOGD],
                                           uint32_t e0) const {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const uint32_t m = mask_of<C>(i);
            uint32_t t = (cnt[i] << (LOGD + E)) + __builtin_popcount(e0 & m);
#pragma unroll
            for (int j = 0; j < LOGD; ++j) t += __builtin_popcount(B[j] & m) << j;
#pragma unroll
            for (int e = 0; e < E; ++e)
                t += (__builtin_popcount(R[e] & m) + __builtin_popcount(P[e] & m)) << (LOGD + e);
            out[i] = t;
        }
    }
};

}  // namespace ppc
