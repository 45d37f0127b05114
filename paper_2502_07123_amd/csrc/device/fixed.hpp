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
    // the 32-bit forms' constants (fx_op_finish on the host)
    int32_t lo, hi;      // saturation bounds -2^(w-1), 2^(w-1) - 1
    int64_t rc;          // 2^(s-1), 0 at s = 0 (the rounding term)
    int32_t ma, mb;      // add: 2^sa, 2^sb (<= 2^30)
};

// The 32-bit forms' constants of an operation.
__host__ __device__ inline FxOp fx_op_finish(FxOp op) {
    op.hi = static_cast<int32_t>((int64_t(1) << (op.w - 1)) - 1);
    op.lo = -op.hi - 1;
    op.rc = op.s > 0 ? int64_t(1) << (op.s - 1) : 0;
    op.ma = int32_t(1) << op.sa;
    op.mb = int32_t(1) << op.sb;
    return op;
}

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

// ---- the same operations on 32-bit words (the kernels' form), without branches on
// the operation's constants.  Operands and results are 32-bit words; the exact
// intermediate is one 64-bit value formed by 32 x 32 -> 64-bit multiply-adds
// (v_mad_i64_i32): a b + rc for a product, a 2^sa + b 2^sb + rc for a sum.  One
// 64-bit arithmetic shift rounds it to the destination's f and two compares against
// the destination's bounds saturate it.  Results and saturation counts equal
// fx_mul / fx_add (tested against them and against the exact rational definition).
__host__ __device__ __forceinline__ int32_t fx32_finish(int64_t x, const FxOp& op, uint32_t& nsat) {
    const int64_t r = x >> op.s;
    const bool below = r < op.lo, above = r > op.hi;
    nsat += (below || above) ? 1u : 0u;
    return below ? op.lo : (above ? op.hi : static_cast<int32_t>(r));
}

__host__ __device__ __forceinline__ int32_t fx32_mul(int32_t a, int32_t b, const FxOp& op, uint32_t& nsat) {
    return fx32_finish(static_cast<int64_t>(a) * b + op.rc, op, nsat);          // |a b| <= 2^62, rc <= 2^61
}

__host__ __device__ __forceinline__ int32_t fx32_add(int32_t a, int32_t b, const FxOp& op, uint32_t& nsat) {
    // |a 2^sa|, |b 2^sb| <= 2^61 and one of sa, sb is 0: no overflow
    return fx32_finish(static_cast<int64_t>(a) * op.ma + static_cast<int64_t>(b) * op.mb + op.rc, op, nsat);
}

}  // namespace mlmc
