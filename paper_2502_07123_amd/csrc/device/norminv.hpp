// Inverse normal CDF of the coupled uniform U = 2^-32 (J + 1/2) (Section 3.1):
// the full-precision increment Z = Phi^-1(U) of the coupled pair (Z, Z~).
//
// FP64: Wichura's algorithm AS 241 (PPND16, Applied Statistics 37, 1988): a
//   rational function of degree 7 in r = 0.180625 - q^2 for |q| = |U - 1/2| <= 0.425,
//   otherwise of r = sqrt(-log(min(U, 1-U))) on [.., 5] and (5, ..].  Relative
//   accuracy about 1e-16.
// FP32: the variable change of Giles ("Approximating the erfinv function", 2011):
//   with y = 2U - 1 and w = -log(4 U (1-U)), Phi^-1 = y P(w) for w < 5 and
//   sign(y) Q(sqrt(w)) beyond, P and Q degree-9 polynomials of this project's own
//   fit (gen_norminv_f32.py); relative error below 3e-7 over the 32-bit grid.
// Both take J directly so that U, 1 - U and U - 1/2 are formed exactly.
#pragma once
#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>

#include "norminv_f32_coeffs.hpp"

namespace mlmc {

__host__ __device__ __forceinline__ double norminv_f64(uint32_t J) {
    // q = U - 1/2 = 2^-32 (J - 2^31 + 1/2): exact
    const int32_t sj = static_cast<int32_t>(J ^ 0x80000000u);
    const double q = (static_cast<double>(sj) + 0.5) * 0x1p-32;
    if (fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        const double num =
            fma(fma(fma(fma(fma(fma(fma(2.5090809287301226727e+3, r, 3.3430575583588128105e+4), r,
                                    6.7265770927008700853e+4), r, 4.5921953931549871457e+4), r,
                            1.3731693765509461125e+4), r, 1.9715909503065514427e+3), r,
                    1.3314166789178437745e+2), r, 3.3871328727963666080e0);
        const double den =
            fma(fma(fma(fma(fma(fma(fma(5.2264952788528545610e+3, r, 2.8729085735721942674e+4), r,
                                    3.9307895800092710610e+4), r, 2.1213794301586595867e+4), r,
                            5.3941960214247511077e+3), r, 6.8718700749205790830e+2), r,
                    4.2313330701600911252e+1), r, 1.0);
        return q * num / den;
    }
    // tail: r = min(U, 1 - U) = 2^-32 (min(J, 2^32-1-J) + 1/2), exact
    const uint32_t v = (J < 0x80000000u) ? J : ~J;
    double r = sqrt(-log((static_cast<double>(v) + 0.5) * 0x1p-32));
    double val;
    if (r <= 5.0) {
        r -= 1.6;
        const double num =
            fma(fma(fma(fma(fma(fma(fma(7.74545014278341407640e-4, r, 2.27238449892691845833e-2), r,
                                    2.41780725177450611770e-1), r, 1.27045825245236838258e0), r,
                            3.64784832476320460504e0), r, 5.76949722146069140550e0), r,
                    4.63033784615654529590e0), r, 1.42343711074968357734e0);
        const double den =
            fma(fma(fma(fma(fma(fma(fma(1.05075007164441684324e-9, r, 5.47593808499534494600e-4), r,
                                    1.51986665636164571966e-2), r, 1.48103976427480074590e-1), r,
                            6.89767334985100004550e-1), r, 1.67638483018380384940e0), r,
                    2.05319162663775882187e0), r, 1.0);
        val = num / den;
    } else {
        r -= 5.0;
        const double num =
            fma(fma(fma(fma(fma(fma(fma(2.01033439929228813265e-7, r, 2.71155556874348757815e-5), r,
                                    1.24266094738807843860e-3), r, 2.65321895265761230930e-2), r,
                            2.96560571828504891230e-1), r, 1.78482653991729133580e0), r,
                    5.46378491116411436990e0), r, 6.65790464350110377720e0);
        const double den =
            fma(fma(fma(fma(fma(fma(fma(2.04426310338993978564e-15, r, 1.42151175831644588870e-7), r,
                                    1.84631831751005468180e-5), r, 7.86869131145613259100e-4), r,
                            1.48753612908506148525e-2), r, 1.36929880922735805310e-1), r,
                    5.99832206555887937690e-1), r, 1.0);
        val = num / den;
    }
    return q < 0.0 ? -val : val;
}

__host__ __device__ __forceinline__ float fast_logf(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __logf(x);
#else
    return logf(x);
#endif
}

__host__ __device__ __forceinline__ float norminv_f32(uint32_t J) {
    using namespace ninv32;
    const int32_t sj = static_cast<int32_t>(J ^ 0x80000000u);
    const float y = (static_cast<float>(sj) + 0.5f) * 0x1p-31f;        // 2U - 1
    const uint32_t v = (J < 0x80000000u) ? J : ~J;
    const float us = (static_cast<float>(v) + 0.5f) * 0x1p-32f;        // min(U, 1-U)
    const float w = -fast_logf((us * (1.0f - us)) * 4.0f);
    if (w < W1) {
        const float t = w - C_MID;
        float p = PC[DEG_C];
#pragma unroll
        for (int k = DEG_C - 1; k >= 0; --k) p = fmaf(p, t, PC[k]);
        return y * p;
    }
    const float t = sqrtf(w) - T_MID;
    float p = PT[DEG_T];
#pragma unroll
    for (int k = DEG_T - 1; k >= 0; --k) p = fmaf(p, t, PT[k]);
    return copysignf(p, y);
}

}  // namespace mlmc
