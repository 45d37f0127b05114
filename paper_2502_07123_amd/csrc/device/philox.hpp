// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox
// S-box on a 128-bit counter with a 64-bit key bumped by Weyl constants.
//
// The paper draws each full-precision uniform from a 32-bit integer J (Section 3,
// notation before 3.1) without naming a generator; counter layout:
//   block b of stream (seed, option, level, estimator) -> counter
//   (b mod 2^32, b div 2^32, level | estimator << 8, option), key = seed.
// In a kernel the last three counter words and the key are wave-uniform, so the
// compiler keeps them (and the first rounds' products on them) in SGPRs.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace mlmc {

struct u32x4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(M0) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(M1) * c.z;
        u32x4 n;
        n.x = static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0;
        n.y = static_cast<uint32_t>(p1);
        n.z = static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1;
        n.w = static_cast<uint32_t>(p0);
        c = n;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

__host__ __device__ __forceinline__ uint32_t stream_c2(int level, int estimator) {
    return (static_cast<uint32_t>(level) & 0xFFu) | ((static_cast<uint32_t>(estimator) & 0xFFu) << 8);
}

}  // namespace mlmc
