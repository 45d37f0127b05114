// Inverse normal CDF of the coupled uniform U = 2^-32 (J + 1/2) (Section 3.1):
// the full-precision increment Z = Phi^-1(U) of the coupled pair (Z, Z~).
//
// Both precisions use the variable change of Giles ("Approximating the erfinv
// function", 2011): with y = 2U - 1 and w = -log(4 U (1-U)), Phi^-1 = y P(w) on a
// central range of w and sign(y) Q(sqrt(w)) beyond, P and Q polynomials of this
// project's own fits.
// FP64: w < 6.25 (all but about 1e-3 of the inputs, so nearly every wave takes one
//   branch), degrees 24 and 20, w from the logarithm log_unit below
//   (gen_norminv_f64.py); relative error below 5e-16 on the 32-bit grid.
// FP32: w < 5, degrees 9 and 9 (gen_norminv_f32.py); relative error below 3e-7.
// Both take J directly so that 2U - 1 (and, in FP32, min(U, 1 - U)) are formed
// exactly.
#pragma once
#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "norminv_f32_coeffs.hpp"
#include "norminv_f64_coeffs.hpp"

namespace mlmc {

// Natural logarithm of x in (0, 1] (the argument 4U(1-U) of w): x = 2^e m with
// m in [1/sqrt 2, sqrt 2), log m = 2 atanh(s) = 2 s + s z Q(z) for s = (m-1)/(m+1),
// z = s^2, Q the atanh series' own coefficients 2/(2k+1) (|s| < 0.172: ten terms
// leave a truncation below 1e-17 relative), and e ln 2 with ln 2 split so that
// e LN2_HI is exact.  Relative error about 3e-16; far cheaper than the general
// library logarithm, which handles every double.
__host__ __device__ __forceinline__ double log_unit(double x) {
    using namespace ninv64;
    int e;
    double m = frexp(x, &e);                      // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;                     // exact
    const double s = f / (2.0 + f);
    const double z = s * s;
    double q = 2.0 / (2 * LOG_TERMS + 1);
#pragma unroll
    for (int k = LOG_TERMS - 1; k >= 1; --k) q = fma(q, z, 2.0 / (2 * k + 1));
    const double lm = fma(s * z, q, 2.0 * s);
    const double de = static_cast<double>(e);
    return fma(de, LN2_HI, fma(de, LN2_LO, lm));
}

#if defined(__HIP_DEVICE_COMPILE__)
// On the device the coefficients are read from constant memory at each use (scalar
// loads into SGPRs) instead of being kept in vector registers across the kernels'
// loops, where they would cost ~90 VGPRs of occupancy.
static __constant__ double g_ninv64_pc[ninv64::DEG_C + 1] = NINV64_PC_INIT;
static __constant__ double g_ninv64_pt[ninv64::DEG_T + 1] = NINV64_PT_INIT;
#define NINV64_PC g_ninv64_pc
#define NINV64_PT g_ninv64_pt
#else
#define NINV64_PC ninv64::PC
#define NINV64_PT ninv64::PT
#endif

// The inverse normal in three parts: the argument (y = 2U - 1, w), the central
// polynomial y P(w - C_MID) and the tail Q(sqrt(w) - T_MID) with y's sign; the value
// is the central one for w < W1, else the tail one.
template <typename T>
struct NinvArg {
    T y, w;
};

// 4U(1-U) = 1 - y^2 exactly, so the fma's single rounding gives the same double as
// rounding us (1 - us) with us = min(U, 1 - U) (1 - us and the scaling by 4 are
// exact), in one instruction instead of the second conversion and three products.
__host__ __device__ __forceinline__ NinvArg<double> ninv64_arg(uint32_t J) {
    const int32_t sj = static_cast<int32_t>(J ^ 0x80000000u);
    const double y = (static_cast<double>(sj) + 0.5) * 0x1p-31;       // 2U - 1, exact
    return NinvArg<double>{y, -log_unit(fma(-y, y, 1.0))};
}

__host__ __device__ __forceinline__ double ninv64_central(const NinvArg<double>& a) {
    using namespace ninv64;
    const double t = a.w - C_MID;
    double p = NINV64_PC[DEG_C];
#pragma unroll
    for (int k = DEG_C - 1; k >= 0; --k) p = fma(p, t, NINV64_PC[k]);
    return a.y * p;
}

__host__ __device__ __forceinline__ double ninv64_tail(const NinvArg<double>& a) {
    using namespace ninv64;
    const double t = sqrt(a.w) - T_MID;
#if defined(__HIP_DEVICE_COMPILE__)
    // The tail runs for about 1e-3 of the inputs: its coefficients are loaded where it
    // runs (the empty asm hides the table's address, so the loads are not hoisted out
    // of the callers' loops), which leaves the loops' scalar registers to the central
    // polynomial instead of spilling them into vector-register lanes.  The address is
    // uniform and the table read-only: through the constant address space the loads
    // are scalar and issued together, one wait instead of one per coefficient pair.
    const double* pg = g_ninv64_pt;
    asm volatile("" : "+s"(pg));
    const __attribute__((address_space(4))) double* pt =
        (const __attribute__((address_space(4))) double*)pg;
#else
    const double* pt = NINV64_PT;
#endif
    double p = pt[DEG_T];
#pragma unroll
    for (int k = DEG_T - 1; k >= 0; --k) p = fma(p, t, pt[k]);
    return copysign(p, a.y);
}

__host__ __device__ __forceinline__ double norminv_f64(uint32_t J) {
    const NinvArg<double> a = ninv64_arg(J);
    return a.w < ninv64::W1 ? ninv64_central(a) : ninv64_tail(a);
}

// Four inverse normals with the same values as norminv_f64: the arguments and the
// central values of all four first, branch-free, so that their dependency chains
// interleave; the rare tail inputs (w >= W1, about 1e-3 of them) are redone after.
__host__ __device__ __forceinline__ void norminv_f64_x4(const uint32_t (&J)[4], double (&Z)[4]) {
    NinvArg<double> a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = ninv64_arg(J[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) Z[i] = ninv64_central(a[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (!(a[i].w < ninv64::W1)) Z[i] = ninv64_tail(a[i]);
}

__host__ __device__ __forceinline__ float fast_logf(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __logf(x);
#else
    return logf(x);
#endif
}

__host__ __device__ __forceinline__ NinvArg<float> ninv32_arg(uint32_t J) {
    const int32_t sj = static_cast<int32_t>(J ^ 0x80000000u);
    const float y = (static_cast<float>(sj) + 0.5f) * 0x1p-31f;        // 2U - 1
    const uint32_t v = (J < 0x80000000u) ? J : ~J;
    const float us = (static_cast<float>(v) + 0.5f) * 0x1p-32f;        // min(U, 1-U)
    return NinvArg<float>{y, -fast_logf((us * (1.0f - us)) * 4.0f)};
}

__host__ __device__ __forceinline__ float ninv32_central(const NinvArg<float>& a) {
    using namespace ninv32;
    const float t = a.w - C_MID;
    float p = PC[DEG_C];
#pragma unroll
    for (int k = DEG_C - 1; k >= 0; --k) p = fmaf(p, t, PC[k]);
    return a.y * p;
}

__host__ __device__ __forceinline__ float ninv32_tail(const NinvArg<float>& a) {
    using namespace ninv32;
    const float t = sqrtf(a.w) - T_MID;
    float p = PT[DEG_T];
#pragma unroll
    for (int k = DEG_T - 1; k >= 0; --k) p = fmaf(p, t, PT[k]);
    return copysignf(p, a.y);
}

__host__ __device__ __forceinline__ float norminv_f32(uint32_t J) {
    const NinvArg<float> a = ninv32_arg(J);
    return a.w < ninv32::W1 ? ninv32_central(a) : ninv32_tail(a);
}

// four FP32 inverse normals, as norminv_f64_x4
__host__ __device__ __forceinline__ void norminv_f32_x4(const uint32_t (&J)[4], float (&Z)[4]) {
    NinvArg<float> a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = ninv32_arg(J[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) Z[i] = ninv32_central(a[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (!(a[i].w < ninv32::W1)) Z[i] = ninv32_tail(a[i]);
}

}  // namespace mlmc
