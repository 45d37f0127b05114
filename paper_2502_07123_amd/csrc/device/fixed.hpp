// Fixed-point operations of the low-precision path (Section 4.1): a variable is a
// two's-complement integer n of w bits with value n 2^-f.  Each operation forms
// its exact result (the 64-bit product, or the sum after exact alignment of the
// operands to the finer f), rounds it once to the destination f -- to nearest,
// ties toward +infinity: (p + 2^(s-1)) >> s -- and saturates it to w bits,
// counting saturations.  Shift amounts are uniform per level and precomputed on
// the host; validation keeps every intermediate below 2^62.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace mlmc {

struct FxOp {
    int32_t sa;   // left shift aligning operand a (add only)
    int32_t sb;   // left shift aligning operand b (add only)
    int32_t s;    // right shift to the destination f (>= 0)
    int32_t w;    // destination word bits
};

__host__ __device__ __forceinline__ int64_t fx_round_shift(int64_t p, int32_t s) {
    return s > 0 ? ((p + (int64_t(1) << (s - 1))) >> s) : p;
}

__host__ __device__ __forceinline__ int64_t fx_saturate(int64_t v, int32_t w, uint32_t& nsat) {
    const int64_t hi = (int64_t(1) << (w - 1)) - 1;
    const int64_t lo = -hi - 1;
    nsat += (v > hi) | (v < lo);
    return v > hi ? hi : (v < lo ? lo : v);
}

// Both factors of every product of the path are saturated variables, table entries or
// quantised constants of at most 32 bits (and Zs = Z + Z' with Z of at most 31 bits),
// so the product is a 32 x 32 -> 64-bit signed multiply.
__host__ __device__ __forceinline__ int64_t fx_mul(int64_t a, int64_t b, const FxOp& op,
                                                   uint32_t& nsat) {
    const int64_t p = static_cast<int64_t>(static_cast<int32_t>(a)) * static_cast<int32_t>(b);
    return fx_saturate(fx_round_shift(p, op.s), op.w, nsat);
}

__host__ __device__ __forceinline__ int64_t fx_add(int64_t a, int64_t b, const FxOp& op,
                                                   uint32_t& nsat) {
    return fx_saturate(fx_round_shift((a << op.sa) + (b << op.sb), op.s), op.w, nsat);
}

}  // namespace mlmc
