// ff_rng.h — Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) for on-device redraws of particles.
// A 128-bit counter is mixed under a 64-bit key by ten rounds of two 32x32->64
// multiplications (multipliers 0xD2511F53 and 0xCD9E8D57) and xors, the key
// advancing by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between rounds.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#else
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace ff {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = 0xD2511F53u * c.x, hi_a = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo_b = 0xCD9E8D57u * c.z, hi_b = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Word w of the stream of draw r of particle g under `seed`: block w/4 of
// Philox with counter (g lo, g hi, r, w/4) and key (seed lo, seed hi).
__device__ __forceinline__ uint32_t draw_word(uint64_t seed, uint64_t g, uint32_t r, int w) {
    const U4 o = philox4x32_10(U4{(uint32_t)g, (uint32_t)(g >> 32), r, (uint32_t)(w >> 2)}, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
    switch (w & 3) {
        case 0: return o.x;
        case 1: return o.y;
        case 2: return o.z;
        default: return o.w;
    }
}

}  // namespace ff
