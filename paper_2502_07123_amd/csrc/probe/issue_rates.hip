// VALU issue rates of the instruction classes the path kernels use, on one GPU:
// eight independent dependency chains per thread, 8 blocks of 256 threads per CU, the
// best of five timed launches.  Printed per class: lane-operations per second and
// wave-instructions per CU per clock (the issue cost of one wave-instruction is the
// reciprocal).  The rates convert the path kernels' SQ instruction counts per class
// into busy issue cycles.  Every LDS index is the top 8 bits of a 32-bit word, below
// the table's 256 entries.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int ITERS = 4096;
constexpr int BLOCK = 256;

__global__ void __launch_bounds__(BLOCK) k_f32_fma(float* out, float seed) {
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-3f + seed + j;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fmaf(a[j], 0.999f, 0.001f);
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) k_i32_xor(uint32_t* out, uint32_t seed) {
    uint32_t a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (threadIdx.x + seed) * (2u * j + 3u);
    const uint32_t k = seed * 7u + 1u;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = (a[j] ^ k) + 0x9E3779B9u * (j + 1);
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s ^= a[j];
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) k_f64_fma(double* out, double seed) {
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-3 + seed + j;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = fma(a[j], 0.999, 0.001);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) k_f64_add(double* out, double seed) {
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 1e-3 + seed + j;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = a[j] + 1e-9 * (j + 1);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

// p <- M lo(p) + p: one widening 32x32->64 multiply-add per step
__global__ void __launch_bounds__(BLOCK) k_u64_mad(uint32_t* out, uint32_t seed) {
    uint64_t p[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) p[j] = uint64_t(threadIdx.x + seed) * (2u * j + 3u) + 1u;
    const uint32_t M = 0xD2511F53u;
    for (int i = 0; i < ITERS; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) p[j] = uint64_t(M) * uint32_t(p[j]) + p[j];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s ^= uint32_t(p[j]) ^ uint32_t(p[j] >> 32);
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

// random 8-byte reads of a 256-entry table (the level-0 sample table's access);
// indices from per-lane Weyl sequences (distinct odd increments), top 8 bits
__global__ void __launch_bounds__(BLOCK) k_lds_b64(double* out, uint32_t seed) {
    __shared__ double tab[256];
    for (int i = threadIdx.x; i < 256; i += BLOCK) tab[i] = i * 1e-3;
    __syncthreads();
    const uint32_t inc = (threadIdx.x * 2654435761u + seed) | 1u;
    uint32_t s0 = inc * 3u, s1 = inc * 7u;
    double acc0 = 0.0, acc1 = 0.0;
    for (int i = 0; i < ITERS; ++i) {
        s0 += inc;
        s1 += inc;
        acc0 += tab[s0 >> 24];
        acc1 += tab[s1 >> 24];
    }
    out[blockIdx.x * BLOCK + threadIdx.x] = acc0 + acc1;
}

// random 4-byte reads of a 256-entry table (an FP16 step table's (Z~, s) pairs)
__global__ void __launch_bounds__(BLOCK) k_lds_b32(float* out, uint32_t seed) {
    __shared__ float tab[256];
    for (int i = threadIdx.x; i < 256; i += BLOCK) tab[i] = i * 1e-3f;
    __syncthreads();
    const uint32_t inc = (threadIdx.x * 2654435761u + seed) | 1u;
    uint32_t s0 = inc * 3u, s1 = inc * 7u;
    float acc0 = 0.0f, acc1 = 0.0f;
    for (int i = 0; i < ITERS; ++i) {
        s0 += inc;
        s1 += inc;
        acc0 += tab[s0 >> 24];
        acc1 += tab[s1 >> 24];
    }
    out[blockIdx.x * BLOCK + threadIdx.x] = acc0 + acc1;
}

// eight independent FP16 multiply-add chains per thread (scalar _Float16)
__global__ void __launch_bounds__(BLOCK) k_f16_fma(_Float16* out, float seed) {
    _Float16 a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = _Float16(seed + threadIdx.x + j);
    const _Float16 m = _Float16(0.999f), c = _Float16(1e-3f);
    for (int i = 0; i < ITERS; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = a[j] * m + c;
    }
    _Float16 s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * BLOCK + threadIdx.x] = s;
}

struct Probe {
    const char* name;
    int insts_per_iter;     // instructions of the class per loop iteration and thread
    int kind;
};

}  // namespace

int main() {
    int cu = 0, clk_khz = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
        hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, 0) != hipSuccess) {
        std::fprintf(stderr, "no HIP device\n");
        return 1;
    }
    std::printf("CUs %d, clock %d kHz\n", cu, clk_khz);
    const int grid = cu * 8;
    void* buf = nullptr;
    if (hipMalloc(&buf, size_t(grid) * BLOCK * 8) != hipSuccess) return 1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1;
    const Probe probes[] = {{"f32_fma", 8, 0}, {"i32_xor_add", 16, 1}, {"f64_fma", 8, 2},
                            {"f64_add", 8, 3}, {"u64_mad", 8, 4},   {"lds_b64_random", 2, 5},
                            {"lds_b32_random", 2, 6}, {"f16_fma", 8, 7}};
    for (const Probe& p : probes) {
        float best = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
            (void)hipEventRecord(a);
            switch (p.kind) {
                case 0: hipLaunchKernelGGL(k_f32_fma, dim3(grid), dim3(BLOCK), 0, 0, (float*)buf, float(rep)); break;
                case 1: hipLaunchKernelGGL(k_i32_xor, dim3(grid), dim3(BLOCK), 0, 0, (uint32_t*)buf, uint32_t(rep)); break;
                case 2: hipLaunchKernelGGL(k_f64_fma, dim3(grid), dim3(BLOCK), 0, 0, (double*)buf, double(rep)); break;
                case 3: hipLaunchKernelGGL(k_f64_add, dim3(grid), dim3(BLOCK), 0, 0, (double*)buf, double(rep)); break;
                case 4: hipLaunchKernelGGL(k_u64_mad, dim3(grid), dim3(BLOCK), 0, 0, (uint32_t*)buf, uint32_t(rep)); break;
                case 5: hipLaunchKernelGGL(k_lds_b64, dim3(grid), dim3(BLOCK), 0, 0, (double*)buf, uint32_t(rep)); break;
                case 6: hipLaunchKernelGGL(k_lds_b32, dim3(grid), dim3(BLOCK), 0, 0, (float*)buf, uint32_t(rep)); break;
                default: hipLaunchKernelGGL(k_f16_fma, dim3(grid), dim3(BLOCK), 0, 0, (_Float16*)buf, float(rep)); break;
            }
            (void)hipEventRecord(b);
            if (hipEventSynchronize(b) != hipSuccess) return 1;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) best = ms;
        }
        const double lane_ops = double(grid) * BLOCK * ITERS * p.insts_per_iter;
        const double per_s = lane_ops / (best * 1e-3);
        const double wave_per_cu_clk = per_s / 64.0 / cu / (clk_khz * 1e3);
        std::printf("%-16s %8.3f ms  %.3e lane-ops/s  %.3f wave-instructions/CU/clk\n", p.name, best, per_s,
                    wave_per_cu_clk);
    }
    (void)hipFree(buf);
    return 0;
}
