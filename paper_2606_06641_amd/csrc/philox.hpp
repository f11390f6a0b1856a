// philox.hpp -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and
// Shaw, SC 2011), device side.  Constants and round structure are the published
// definition, so outputs match its known-answer vectors.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace afs {
namespace dev {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox_round(U4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t lo0 = m0 * c.x, hi0 = __umulhi(m0, c.x);
    const uint32_t lo1 = m1 * c.z, hi1 = __umulhi(m1, c.z);
    return U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        c = philox_round(c, k0, k1);
    }
    return c;
}

// A multiple of 2^-23 in [-1, 1) from the top 24 bits of a word (exact in FP32).
__device__ __forceinline__ float philox_pm1(uint32_t word)
{
    return (float)(word >> 8) * 0x1p-23f - 1.0f;
}

}  // namespace dev
}  // namespace afs
