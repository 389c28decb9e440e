// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), for device and host:
// ten rounds on a 4-word counter with a 2-word key.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace wdr {

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

__host__ __device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c[0], hi0 = mulhi64(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = mulhi64(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// 53-bit uniform in (0, 1) from a Philox word
__host__ __device__ inline double uniform53(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

}  // namespace wdr
