// The exact normal of the coupled pair, Z = Phi^-1(U) with U = 2^-32 (J + 1/2)
// (Section 3.1), exposed on its own so that the device and host builds of the path
// kernels' inverse normals can be checked against high-precision quantiles.  The
// device entry evaluates four words per thread with the four-wide form that the
// exact-normal loops use (norminv_*_x4) and a ragged tail with the scalar form.
#include <hip/hip_runtime.h>

#include <string>

#include "device/norminv.hpp"
#include "runtime.hpp"

namespace mlmc {

template <bool F32>
__global__ void __launch_bounds__(256) k_inverse_normal(const uint32_t* __restrict__ J, uint64_t n,
                                                        void* __restrict__ out) {
    using ZT = typename std::conditional<F32, float, double>::type;
    ZT* z = static_cast<ZT*>(out);
    const uint64_t i = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
    if (i >= n) return;
    if (i + 4 <= n) {
        const uint32_t w[4] = {J[i], J[i + 1], J[i + 2], J[i + 3]};
        ZT r[4];
        if constexpr (F32) norminv_f32_x4(w, r);
        else norminv_f64_x4(w, r);
#pragma unroll
        for (int k = 0; k < 4; ++k) z[i + k] = r[k];
    } else {
        for (uint64_t k = i; k < n; ++k) z[k] = F32 ? ZT(norminv_f32(J[k])) : ZT(norminv_f64(J[k]));
    }
}

}  // namespace mlmc

using namespace mlmc;

extern "C" mlmc_status mlmc_inverse_normal(mlmc_context* ctx, const uint32_t* J_dev, uint64_t n,
                                           int32_t arith, void* out_dev) {
    if (!ctx) return MLMC_E_INVALID;
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    if (arith != MLMC_ARITH_FP64 && arith != MLMC_ARITH_FP32)
        return fail(ctx, MLMC_E_INVALID, "mlmc_inverse_normal: arith must be FP64 or FP32");
    if (n == 0) return MLMC_OK;
    if (!J_dev || !out_dev) return fail(ctx, MLMC_E_INVALID, "mlmc_inverse_normal: NULL buffer");
    const uint64_t threads = (n + 3) / 4;
    if (threads > uint64_t(0xFFFFFFFFu) * 256u) return fail(ctx, MLMC_E_INVALID, "mlmc_inverse_normal: n too large");
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    hipError_t e = hipSetDevice(ctx->device);
    const dim3 grid(static_cast<uint32_t>((threads + 255) / 256));
    if (e == hipSuccess) {
        if (arith == MLMC_ARITH_FP32)
            hipLaunchKernelGGL(k_inverse_normal<true>, grid, dim3(256), 0, ctx->stream, J_dev, n, out_dev);
        else
            hipLaunchKernelGGL(k_inverse_normal<false>, grid, dim3(256), 0, ctx->stream, J_dev, n, out_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("mlmc_inverse_normal: ") + hipGetErrorString(e));
    return MLMC_OK;
}

extern "C" mlmc_status mlmc_inverse_normal_host(const uint32_t* J, uint64_t n, int32_t arith, void* out) {
    if (arith != MLMC_ARITH_FP64 && arith != MLMC_ARITH_FP32) return MLMC_E_INVALID;
    if (n && (!J || !out)) return MLMC_E_INVALID;
    if (arith == MLMC_ARITH_FP32) {
        float* z = static_cast<float*>(out);
        for (uint64_t i = 0; i < n; ++i) z[i] = norminv_f32(J[i]);
    } else {
        double* z = static_cast<double*>(out);
        for (uint64_t i = 0; i < n; ++i) z[i] = norminv_f64(J[i]);
    }
    return MLMC_OK;
}
