// Sensitivities of the rounding-error model (Section 4.2) on the GPU.
//
// For one level l of the European call, every path is run twice in FP64 with exact
// normals from the correction estimator's stream (the exact side of Section 2.2):
// the first pass finds the payoff derivatives G_f = 1[X_N > k] and
// G_c = -1[Xc > k]; the second pass repeats the path and forms the adjoint of every
// variable instance of Algorithm 1 (Milstein per R3) in the forward order.  GBM makes
// the reverse sweep closed-form: X_{n+1} = X_n (1 + s_n), so
//   dP/dX_{n+1} = G X_N / X_{n+1},   dP/dmul2_n = dP/dX_{n+1},   dP/ds_n = dP/dX_{n+1} X_n,
// and the adjoints of s_n's chain (sum2, mul3, zm1, zsq, sum1, mul1, the constants and
// the normal) follow from dP/ds_n by the chain rule.  A coarse step uses
// Zs = Z_2m + Z_2m+1, so the adjoint of a fine normal adds its coarse step's term.
//
// Per (variable, instance) the squared adjoints are summed over paths: a wave sums
// its 64 lanes by cross-lane shuffles and one lane adds the result to a global FP64
// accumulator (atomic).  Per variable the largest |value| over all instances sets
// its exponent (Section 4.1).  The host turns the sums into
//   S_v = sum_j E[xbar_vj^2],  R_v = sum_j sqrt(E[xbar_vj^2]).
// Instance numbering: fine step n -> j = n, coarse step m -> j = N + m; Z: the fine
// normals j = n; con1: j = 0 (fine), 1 (coarse, con1c); con2, con3: j = 0.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "device/norminv.hpp"
#include "device/philox.hpp"
#include "host/prepare.hpp"
#include "runtime.hpp"

namespace mlmc {
namespace {

struct SensParams {
    double con1, con1c, con2, con3, k;
    uint64_t n_paths, path_begin;
    uint32_t c2, c3, k0, k1;
    int32_t level, mil;
    uint32_t ni;                    // instances per variable in the accumulator (3N/2; level 0: 1)
    uint32_t pad;
};

constexpr int NV = MLMC_NVARS;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// adds the wave's sum of x^2 (x = 0 on idle lanes) to acc[v * ni + j]
__device__ __forceinline__ void record(double* acc, const SensParams& P, int v, uint32_t j, double x) {
    const double s = wave_sum(x * x);
    if ((threadIdx.x & 63) == 0) atomicAdd(&acc[static_cast<size_t>(v) * P.ni + j], s);
}

// uniform word of stream position (path, step)
__device__ __forceinline__ uint32_t word_at(const SensParams& P, uint64_t path, uint32_t n) {
    const uint64_t pos = (path << P.level) + n;
    const uint64_t b = pos >> 2;
    const u32x4 r = philox4x32_10(u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), P.c2, P.c3},
                                  P.k0, P.k1);
    switch (pos & 3) {
        case 0: return r.x;
        case 1: return r.y;
        case 2: return r.z;
        default: return r.w;
    }
}

struct Chain {
    double mul1, sum1, zsq, zm1, mul3, sum2, s;
};

__device__ __forceinline__ Chain chain(const SensParams& P, double z, double c1, double cz) {
    Chain c;
    c.mul1 = P.con2 * z;
    c.sum1 = c1 + c.mul1;
    if (P.mil) {
        c.zsq = z * z;
        c.zm1 = c.zsq - cz;
        c.mul3 = P.con3 * c.zm1;
        c.sum2 = c.sum1 + c.mul3;
        c.s = c.sum2;
    } else {
        c.zsq = c.zm1 = c.mul3 = c.sum2 = 0.0;
        c.s = c.sum1;
    }
    return c;
}

// Grid-stride over whole waves of paths, so every lane of a wave runs the same
// steps (the shuffles need all 64 lanes); lanes past the end contribute zeros.
__global__ void __launch_bounds__(256) k_sens(SensParams P, double* acc, unsigned long long* maxabs,
                                              double* moments) {
    const uint32_t N = 1u << P.level;
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
    double mx[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) mx[v] = 0.0;
    double m1 = 0.0, m2 = 0.0;
    for (uint64_t w0 = wave * 64; w0 < P.n_paths; w0 += n_waves * 64) {
        const bool valid = w0 + lane < P.n_paths;
        const uint64_t path = P.path_begin + (valid ? w0 + lane : 0);
        const double on = valid ? 1.0 : 0.0;
        // pass 1: terminal values
        double X = 1.0, Xc = 1.0;
        for (uint32_t n = 0; n < N; n += 2) {
            const double z0 = norminv_f64(word_at(P, path, n));
            const double s0 = chain(P, z0, P.con1, 1.0).s;
            X = X + X * s0;
            if (N == 1) break;
            const double z1 = norminv_f64(word_at(P, path, n + 1));
            const double s1 = chain(P, z1, P.con1, 1.0).s;
            X = X + X * s1;
            const double sc = chain(P, z0 + z1, P.con1c, 2.0).s;
            Xc = Xc + Xc * sc;
        }
        const double XN = X, XcN = Xc;
        const double Gf = XN > P.k ? on : 0.0;
        const double Gc = (P.level >= 1 && XcN > P.k) ? -on : 0.0;
        const double dP = (fmax(XN - P.k, 0.0) - (P.level >= 1 ? fmax(XcN - P.k, 0.0) : 0.0)) * on;
        m1 += dP;
        m2 += dP * dP;
        // pass 2: adjoints in the forward order
        double c1f = 0.0, c1c = 0.0, c2b = 0.0, c3b = 0.0;
        X = 1.0;
        Xc = 1.0;
        for (uint32_t n = 0; n < N; n += 2) {
            double zf[2], zb[2];
            const int steps = N == 1 ? 1 : 2;
            for (int t = 0; t < steps; ++t) {
                const double z = norminv_f64(word_at(P, path, n + t));
                zf[t] = z;
                const Chain c = chain(P, z, P.con1, 1.0);
                const double mul2 = X * c.s;
                const double Xn = X + mul2;
                const double xb = Gf * XN / Xn;              // dP/dX_{n+1}
                const double sb = xb * X;                    // dP/ds_n
                const uint32_t j = n + t;
                record(acc, P, MLMC_V_X, j, xb);
                record(acc, P, MLMC_V_MUL2, j, xb);
                record(acc, P, MLMC_V_SUM1, j, sb);
                record(acc, P, MLMC_V_MUL1, j, sb);
                double zbt = sb * P.con2;
                c1f += sb;
                c2b += sb * z;
                if (P.mil) {
                    const double zmb = sb * P.con3;
                    record(acc, P, MLMC_V_SUM2, j, sb);
                    record(acc, P, MLMC_V_MUL3, j, sb);
                    record(acc, P, MLMC_V_ZM1, j, zmb);
                    record(acc, P, MLMC_V_ZSQ, j, zmb);
                    c3b += sb * c.zm1;
                    zbt += 2.0 * z * zmb;
                    mx[MLMC_V_ZSQ] = fmax(mx[MLMC_V_ZSQ], fabs(c.zsq) * on);
                    mx[MLMC_V_ZM1] = fmax(mx[MLMC_V_ZM1], fabs(c.zm1) * on);
                    mx[MLMC_V_MUL3] = fmax(mx[MLMC_V_MUL3], fabs(c.mul3) * on);
                    mx[MLMC_V_SUM2] = fmax(mx[MLMC_V_SUM2], fabs(c.sum2) * on);
                }
                zb[t] = zbt;
                mx[MLMC_V_MUL1] = fmax(mx[MLMC_V_MUL1], fabs(c.mul1) * on);
                mx[MLMC_V_SUM1] = fmax(mx[MLMC_V_SUM1], fabs(c.sum1) * on);
                mx[MLMC_V_MUL2] = fmax(mx[MLMC_V_MUL2], fabs(mul2) * on);
                mx[MLMC_V_X] = fmax(mx[MLMC_V_X], fabs(Xn) * on);
                X = Xn;
            }
            if (N == 1) {
                record(acc, P, MLMC_V_Z, 0, zb[0]);
                break;
            }
            // the coarse step of this fine pair
            const double zs = zf[0] + zf[1];
            const Chain c = chain(P, zs, P.con1c, 2.0);
            const double mul2 = Xc * c.s;
            const double Xn = Xc + mul2;
            const double xb = Gc * XcN / Xn;
            const double sb = xb * Xc;
            const uint32_t j = N + n / 2;
            record(acc, P, MLMC_V_X, j, xb);
            record(acc, P, MLMC_V_MUL2, j, xb);
            record(acc, P, MLMC_V_SUM1, j, sb);
            record(acc, P, MLMC_V_MUL1, j, sb);
            double zbc = sb * P.con2;
            c1c += sb;
            c2b += sb * zs;
            if (P.mil) {
                const double zmb = sb * P.con3;
                record(acc, P, MLMC_V_SUM2, j, sb);
                record(acc, P, MLMC_V_MUL3, j, sb);
                record(acc, P, MLMC_V_ZM1, j, zmb);
                record(acc, P, MLMC_V_ZSQ, j, zmb);
                c3b += sb * c.zm1;
                zbc += 2.0 * zs * zmb;
                mx[MLMC_V_ZSQ] = fmax(mx[MLMC_V_ZSQ], fabs(c.zsq) * on);
                mx[MLMC_V_ZM1] = fmax(mx[MLMC_V_ZM1], fabs(c.zm1) * on);
                mx[MLMC_V_MUL3] = fmax(mx[MLMC_V_MUL3], fabs(c.mul3) * on);
                mx[MLMC_V_SUM2] = fmax(mx[MLMC_V_SUM2], fabs(c.sum2) * on);
            }
            mx[MLMC_V_MUL1] = fmax(mx[MLMC_V_MUL1], fabs(c.mul1) * on);
            mx[MLMC_V_SUM1] = fmax(mx[MLMC_V_SUM1], fabs(c.sum1) * on);
            mx[MLMC_V_MUL2] = fmax(mx[MLMC_V_MUL2], fabs(mul2) * on);
            mx[MLMC_V_X] = fmax(mx[MLMC_V_X], fabs(Xn) * on);
            Xc = Xn;
            record(acc, P, MLMC_V_Z, n, zb[0] + zbc);
            record(acc, P, MLMC_V_Z, n + 1, zb[1] + zbc);
        }
        record(acc, P, MLMC_V_CON1, 0, c1f);
        if (P.level >= 1) record(acc, P, MLMC_V_CON1, 1, c1c);
        record(acc, P, MLMC_V_CON2, 0, c2b);
        if (P.mil) record(acc, P, MLMC_V_CON3, 0, c3b);
    }
    // exponents and the level's moments
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double m = wave_max(mx[v]);
        if (lane == 0 && m > 0.0) atomicMax(&maxabs[v], static_cast<unsigned long long>(__double_as_longlong(m)));
    }
    m1 = wave_sum(m1);
    m2 = wave_sum(m2);
    if (lane == 0) {
        atomicAdd(&moments[0], m1);
        atomicAdd(&moments[1], m2);
    }
}

}  // namespace
}  // namespace mlmc

using namespace mlmc;

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        const hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, MLMC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" mlmc_status mlmc_error_model_compute(mlmc_context* ctx, const mlmc_problem* prob, int32_t level,
                                                uint64_t n_paths, int32_t q, uint64_t seed, uint32_t option_id,
                                                mlmc_error_model* out) {
    if (!ctx || !prob || !out) return MLMC_E_INVALID;
    if (out->struct_size != sizeof(mlmc_error_model)) return fail(ctx, MLMC_E_VERSION, "mlmc_error_model.struct_size mismatch");
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    if (ctx->ws_held) return fail(ctx, MLMC_E_BUSY, "a running server's sweep engine holds the workspace");
    std::string err;
    mlmc_status s = validate_problem(prob, err);
    if (s != MLMC_OK) return fail(ctx, s, err);
    if (prob->payoff_mask != (1u << MLMC_PAY_EURO))
        return fail(ctx, MLMC_E_INVALID, "the error model is for the European call alone");
    if (level < 0 || level > 20 || n_paths < 2 || q < 1 || q > 16)
        return fail(ctx, MLMC_E_INVALID, "need 0 <= level <= 20, n_paths >= 2, 1 <= q <= 16");
    if (n_paths > (UINT64_MAX >> level)) return fail(ctx, MLMC_E_INVALID, "paths x 2^level exceeds the stream");
    const uint32_t N = 1u << level;
    SensParams P;
    std::memset(&P, 0, sizeof(P));
    const double h = prob->T / static_cast<double>(N);
    P.con1 = prob->r * h;
    P.con1c = prob->r * (2.0 * h);
    P.con2 = prob->sigma * std::sqrt(h);
    P.con3 = ((0.5 * prob->sigma) * prob->sigma) * h;
    P.k = prob->K / prob->S0;
    P.n_paths = n_paths;
    P.path_begin = 0;
    P.c2 = stream_c2(level, MLMC_EST_CORR);
    P.c3 = option_id;
    P.k0 = static_cast<uint32_t>(seed);
    P.k1 = static_cast<uint32_t>(seed >> 32);
    P.level = level;
    P.mil = prob->scheme == MLMC_MILSTEIN ? 1 : 0;
    P.ni = level >= 1 ? N + N / 2 : 1;
    const size_t acc_n = static_cast<size_t>(NV) * P.ni;
    const size_t bytes = acc_n * 8 + NV * 8 + 2 * 8;

    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    s = drain_flights(ctx);                 // the workspace is needed whole
    if (s != MLMC_OK) return s;
    if (bytes > ctx->ws_bytes) return fail(ctx, MLMC_E_NOMEM, "workspace too small for the accumulators");
    HIPCHK(hipSetDevice(ctx->device));
    double* acc = reinterpret_cast<double*>(ctx->ws);
    unsigned long long* maxabs = reinterpret_cast<unsigned long long*>(ctx->ws + acc_n * 8);
    double* moments = reinterpret_cast<double*>(ctx->ws + acc_n * 8 + NV * 8);
    HIPCHK(hipMemsetAsync(ctx->ws, 0, bytes, ctx->stream));
    const uint64_t waves = (n_paths + 63) / 64;
    const uint32_t cap = static_cast<uint32_t>(std::max(1, ctx->cu_count)) * 8;
    const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(cap, (waves + 3) / 4));
    hipLaunchKernelGGL(k_sens, dim3(grid), dim3(256), 0, ctx->stream, P, acc, maxabs, moments);
    HIPCHK(hipGetLastError());
    std::vector<uint8_t> host(bytes);
    HIPCHK(hipMemcpyAsync(host.data(), ctx->ws, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));

    const double* A = reinterpret_cast<const double*>(host.data());
    std::memset(out, 0, sizeof(*out));
    out->struct_size = sizeof(mlmc_error_model);
    out->level = level;
    out->scheme = prob->scheme;
    out->table_bits = q;
    out->n_paths = n_paths;
    const double inv = 1.0 / static_cast<double>(n_paths);
    for (int v = 0; v < NV; ++v) {
        const bool mil_only = v == MLMC_V_CON3 || v == MLMC_V_ZSQ || v == MLMC_V_ZM1 || v == MLMC_V_MUL3 ||
                              v == MLMC_V_SUM2;
        out->used[v] = (!mil_only || P.mil) ? 1 : 0;
        if (!out->used[v]) continue;
        uint32_t count;
        if (v == MLMC_V_Z) count = N;
        else if (v == MLMC_V_CON1) count = level >= 1 ? 2 : 1;
        else if (v == MLMC_V_CON2 || v == MLMC_V_CON3) count = 1;
        else count = level >= 1 ? N + N / 2 : 1;
        double S = 0.0, R = 0.0;
        for (uint32_t j = 0; j < count; ++j) {
            const double m2 = A[static_cast<size_t>(v) * P.ni + j] * inv;
            S += m2;
            R += std::sqrt(m2);
        }
        out->S[v] = S;
        out->R[v] = R;
    }
    // exponents: |x| < 2^e over every instance (Section 4.1); the constants' own
    // values; Z's from the table the kernel quantises (its largest |T_q[k]|)
    uint64_t bits[NV];
    std::memcpy(bits, host.data() + acc_n * 8, sizeof(bits));
    double mx[NV];
    for (int v = 0; v < NV; ++v) std::memcpy(&mx[v], &bits[v], 8);
    mx[MLMC_V_CON1] = std::max(std::fabs(P.con1), level >= 1 ? std::fabs(P.con1c) : 0.0);
    mx[MLMC_V_CON2] = std::fabs(P.con2);
    mx[MLMC_V_CON3] = std::fabs(P.con3);
    mx[MLMC_V_Z] = table_max_abs(q);
    for (int v = 0; v < NV; ++v) {
        if (!out->used[v]) continue;
        int e = 0;
        if (mx[v] > 0.0) std::frexp(mx[v], &e);
        else e = -1074;
        out->e[v] = e;
    }
    const double* mom = reinterpret_cast<const double*>(host.data() + acc_n * 8 + NV * 8);
    const double n = static_cast<double>(n_paths);
    out->V_level = (mom[1] - mom[0] * mom[0] / n) / (n - 1.0);
    out->mse = table_mse(q);
    return MLMC_OK;
}
