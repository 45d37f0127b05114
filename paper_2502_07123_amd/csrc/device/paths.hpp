// Per-thread work of the path kernels: one "path group" of coupled fine/coarse
// GBM paths (Section 2.1; Algorithm 1), its payoffs and the estimator samples
// (Section 2.2), accumulated into per-thread sums.
//
// Steps.  Exact side (FP64, or FP32 for the plain-FP32 estimator):
//   s = con1 + con2 Z (+ con3 (Z^2 - 1), Milstein),  X <- X + X s
//   coarse, once per fine pair: Zs = Z_2m + Z_2m+1, s = con1c + con2 Zs
//   (+ con3 (Zs^2 - 2)), Xc <- Xc + Xc s  (drift and volatility frozen over the
//   pair, Section 2.1).
// Low-precision side with Method-1 normals (Section 3.1).  The table holds, per
// interval k, (Z~_k, s_k) with s_k the step multiplier the arithmetic would form
// from Z~_k -- a function of k alone -- so the fine step is X <- X + X s_k:
//   FP32 / FP16:  s_k is Algorithm 1's multiplier chain evaluated on Z~_k with each
//          operation rounded to the side's type (built on the host); the coarse
//          step runs the same chain on Zs = Z~_a + Z~_b.  Bit-exact by construction.
//   FIXED: s_k is sum1 (Euler) or sum2 (Milstein) of Algorithm 1's chain in the
//          per-variable formats, built on the host with the same rounding; the
//          coarse step runs the whole chain on Zs.  Bit-exact by construction.
// Uniforms: Philox block b of the stream gives 4 words; unpacked, each word is one
// step (index = top q bits, exact normal from the whole word); packed (APPROX), a
// word holds F = floor(32/q) indices, field j = bits [32-q(j+1), 32-qj).
#pragma once
#include <cmath>
#include <cstdint>
#include <hip/hip_runtime.h>
#include <type_traits>

#include "../common.hpp"
#include "fixed.hpp"
#include "norminv.hpp"
#include "philox.hpp"

namespace mlmc {

template <int NP>
struct Acc {
    double s1[NP], s2[NP], e1[NP], e2[NP];
    int64_t i1[NP];
    uint64_t i2lo[NP], i2hi[NP];
    uint32_t n, sat, nonfinite;
};

template <int NP>
__host__ __device__ __forceinline__ void acc_zero(Acc<NP>& a) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        a.s1[p] = a.s2[p] = a.e1[p] = a.e2[p] = 0.0;
        a.i1[p] = 0;
        a.i2lo[p] = a.i2hi[p] = 0;
    }
    a.n = a.sat = a.nonfinite = 0;
}

// ----------------------------------------------------------------- float sides
template <typename T>
struct FSide {
    T xf, xc, af, ac, mf, mc, zp, sp;

    __host__ __device__ __forceinline__ void init() {
        xf = xc = mf = mc = T(1);
        af = ac = T(0);
        zp = sp = T(0);
    }
    __host__ __device__ __forceinline__ void track_f(bool on) {
        if (on) { af = af + xf; mf = xf < mf ? xf : mf; }
    }
    __host__ __device__ __forceinline__ void track_c(bool on) {
        if (on) { ac = ac + xc; mc = xc < mc ? xc : mc; }
    }
    // payoff p of the fine (coarse) path with log2 of its step count m
    __host__ __device__ __forceinline__ T payoff(int p, bool fine, int m, T k, T b) const {
#pragma clang fp contract(off)
        const T X = fine ? xf : xc;
        const T zero = T(0);
        switch (p) {
            case MLMC_PAY_FORWARD: return X;
            case MLMC_PAY_EURO: { const T d = X - k; return d > zero ? d : zero; }
            case MLMC_PAY_ASIAN: {
                T t = (fine ? af : ac) - T(0.5) * X;
                t = t + T(0.5);                                  // + X_0 / 2, X_0 = 1
                const T A = t * T(ldexp(1.0, -m));
                const T d = A - k;
                return d > zero ? d : zero;
            }
            case MLMC_PAY_BARRIER: {
                const T d = X - k;
                return ((fine ? mf : mc) > b && d > zero) ? d : zero;
            }
            default: return X > k ? k : zero;                    // digital
        }
    }
};

// exact-normal step in FP64 or FP32
template <bool MIL>
__host__ __device__ __forceinline__ void exact_step(FSide<double>& s, double Z, const LevelDev& L,
                                                    bool coarse_on, bool odd, bool track) {
    double t = fma(L.con2, Z, L.con1);
    if (MIL) t = fma(L.con3, fma(Z, Z, -1.0), t);
    s.xf = fma(s.xf, t, s.xf);
    s.track_f(track);
    if (coarse_on) {
        if (!odd) {
            s.zp = Z;
        } else {
            const double zs = s.zp + Z;
            double tc = fma(L.con2, zs, L.con1c);
            if (MIL) tc = fma(L.con3, fma(zs, zs, -2.0), tc);
            s.xc = fma(s.xc, tc, s.xc);
            s.track_c(track);
        }
    }
}

// Low-precision float steps (FP32, FP16) follow Algorithm 1 operation by operation,
// each rounded to the side's type (no fused multiply-add), so the paths are
// reproducible bit for bit.  The multiplier of one step from a normal z:
// mul1 = con2 z, sum1 = con1 + mul1 (Milstein: zsq = z z, zm1 = zsq - c,
// mul3 = con3 zm1, sum2 = sum1 + mul3).
template <bool MIL, typename T>
__host__ __device__ __forceinline__ T multiplier_lp(T z, T con1, T con2, T con3, T c) {
#pragma clang fp contract(off)
    const T mul1 = con2 * z;
    T s = con1 + mul1;
    if (MIL) {
        const T zsq = z * z;
        const T zm1 = zsq - c;
        const T mul3 = con3 * zm1;
        s = s + mul3;
    }
    return s;
}

// two binary16 values, operated on as packed math on the device (v_pk_*_f16)
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

#if defined(__HIP_DEVICE_COMPILE__)
// FP16 on the device: the coarse step's independent operation pairs as packed math,
// (mul1, zsq) = (con2, zs) * (zs, zs) and (sum1, zm1) = (con1, -c) + (mul1, zsq), each
// lane rounded as the scalar operation (IEEE, per element), so the result equals
// multiplier_lp<MIL, _Float16> bit for bit.
template <bool MIL>
__device__ __forceinline__ _Float16 multiplier_h2(_Float16 z, _Float16 con1, _Float16 con2, _Float16 con3,
                                                  _Float16 c) {
#pragma clang fp contract(off)
    if (!MIL) return con1 + con2 * z;
    const half2v p = half2v{con2, z} * half2v{z, z};            // v_pk_mul_f16
    const half2v q = half2v{con1, -c} + p;                      // v_pk_add_f16
    const _Float16 mul3 = con3 * q.y;
    return q.x + mul3;
}
#endif

template <typename T>
__host__ __device__ __forceinline__ T advance_lp(T x, T s) {
#pragma clang fp contract(off)
    const T mul2 = x * s;
    return x + mul2;
}

template <bool MIL>
__host__ __device__ __forceinline__ float multiplier32(float z, float con1, float con2, float con3,
                                                       float c) {
    return multiplier_lp<MIL, float>(z, con1, con2, con3, c);
}
__host__ __device__ __forceinline__ float advance32(float x, float s) { return advance_lp<float>(x, s); }

// The low-precision side's constants in its own type.
template <typename T>
struct LpConst {
    T con1, con1c, con2, con3, k, b;
};
template <typename T>
__host__ __device__ __forceinline__ LpConst<T> lp_const(const LevelDev& L);
template <>
__host__ __device__ __forceinline__ LpConst<float> lp_const<float>(const LevelDev& L) {
    return LpConst<float>{L.fcon1, L.fcon1c, L.fcon2, L.fcon3, L.fk, L.fb};
}
template <>
__host__ __device__ __forceinline__ LpConst<_Float16> lp_const<_Float16>(const LevelDev& L) {
    return LpConst<_Float16>{L.hcon1, L.hcon1c, L.hcon2, L.hcon3, L.hk, L.hb};
}

// A step-table entry of a float side: (Z~_k, s_k) in the side's type.
template <typename T>
struct TabPair {
    T z, s;
};

template <bool MIL>
__host__ __device__ __forceinline__ void exact_step(FSide<float>& s, float Z, const LevelDev& L,
                                                    bool coarse_on, bool odd, bool track) {
    s.xf = advance32(s.xf, multiplier32<MIL>(Z, L.fcon1, L.fcon2, L.fcon3, 1.0f));
    s.track_f(track);
    if (coarse_on) {
        if (!odd) {
            s.zp = Z;
        } else {
            const float zs = s.zp + Z;
            s.xc = advance32(s.xc, multiplier32<MIL>(zs, L.fcon1c, L.fcon2, L.fcon3, 2.0f));
            s.track_c(track);
        }
    }
}

// table step, float low-precision side; entry = (Z~_k, s_k) with s_k the fine
// multiplier of Z~_k (multiplier_lp evaluated on the host)
template <bool MIL, typename T>
__host__ __device__ __forceinline__ void table_step(FSide<T>& s, T z, T sk, const LevelDev& L,
                                                    bool coarse_on, bool odd, bool track) {
    s.xf = advance_lp<T>(s.xf, sk);
    s.track_f(track);
    if (coarse_on) {
        if (!odd) {
            s.zp = z;
        } else {
#pragma clang fp contract(off)
            const LpConst<T> c = lp_const<T>(L);
            const T zs = s.zp + z;
#if defined(__HIP_DEVICE_COMPILE__)
            if constexpr (std::is_same<T, _Float16>::value)
                s.xc = advance_lp<T>(s.xc, multiplier_h2<MIL>(zs, c.con1c, c.con2, c.con3, T(2)));
            else
#endif
                s.xc = advance_lp<T>(s.xc, multiplier_lp<MIL, T>(zs, c.con1c, c.con2, c.con3, T(2)));
            s.track_c(track);
        }
    }
}

// ----------------------------------------------------------------- fixed side
// Path variables are 32-bit words (saturated to their w <= 32 bits); the Asian sums
// of X over the grid are exact 64-bit integers.
struct XSide {
    int32_t xf, xc, mf, mc, zp;
    int64_t af, ac;
    uint32_t nsat;

    __host__ __device__ __forceinline__ void init(const LevelDev& L) {
        xf = xc = mf = mc = static_cast<int32_t>(int64_t(1) << L.fX);
        af = ac = 0;
        zp = 0;
        nsat = 0;
    }
    __host__ __device__ __forceinline__ int64_t payoff(int p, bool fine, int m,
                                                       const LevelDev& L) {
        const int64_t X = fine ? xf : xc;
        switch (p) {
            case MLMC_PAY_FORWARD: return X;
            case MLMC_PAY_EURO: { const int64_t d = X - L.ik; return d > 0 ? d : 0; }
            case MLMC_PAY_ASIAN: {
                // 2 * trapezoid sum = 2 sum_{n=1..N} X_n - X_N + X_0, exact; / 2^(m+1)
                const int64_t s2 = 2 * (fine ? af : ac) - X + (int64_t(1) << L.fX);
                const int64_t A = fx_saturate(fx_round_shift(s2, m + 1), L.wX, nsat);
                const int64_t d = A - L.ik;
                return d > 0 ? d : 0;
            }
            case MLMC_PAY_BARRIER: {
                const int64_t d = X - L.ik;
                return ((fine ? mf : mc) > L.ib && d > 0) ? d : 0;
            }
            default: return X > L.ik ? L.ik : 0;
        }
    }
};

// Algorithm 1's fine step X <- X + X s_k (s_k tabulated per index) and, once per
// fine pair, the coarse chain on Zs = Z_2m + Z_2m+1, every operation in the 32-bit
// forms of device/fixed.hpp.
template <bool MIL>
__host__ __device__ __forceinline__ void fixed_step(XSide& s, int32_t z, int32_t sk,
                                                    const LevelDev& L, bool coarse_on, bool odd,
                                                    bool track) {
    const int32_t m2 = fx32_mul(s.xf, sk, L.op_mul2, s.nsat);
    s.xf = fx32_add(s.xf, m2, L.op_addX, s.nsat);
    if (track) { s.af += s.xf; s.mf = s.xf < s.mf ? s.xf : s.mf; }
    if (coarse_on) {
        if (!odd) {
            s.zp = z;
        } else {
            const int32_t zs = s.zp + z;                       // exact: Z has at most 31 bits
            const int32_t m1 = fx32_mul(static_cast<int32_t>(L.icon2), zs, L.op_mul1, s.nsat);
            int32_t sc = fx32_add(static_cast<int32_t>(L.icon1c), m1, L.op_sum1, s.nsat);
            if (MIL) {
                const int32_t zq = fx32_mul(zs, zs, L.op_zsq, s.nsat);
                const int32_t zm = fx32_add(zq, static_cast<int32_t>(-L.izm_c2), L.op_zm1, s.nsat);
                const int32_t m3 = fx32_mul(static_cast<int32_t>(L.icon3), zm, L.op_mul3, s.nsat);
                sc = fx32_add(sc, m3, L.op_sum2, s.nsat);
            }
            const int32_t m2c = fx32_mul(s.xc, sc, L.op_mul2, s.nsat);
            s.xc = fx32_add(s.xc, m2c, L.op_addX, s.nsat);
            if (track) { s.ac += s.xc; s.mc = s.xc < s.mc ? s.xc : s.mc; }
        }
    }
}

// ------------------------------------------------------------- path kernel body
// EST: MLMC_EST_*; ARITH: arithmetic of the table side (APPROX/CORR) or of the
// plain side (PLAIN: FP64 or FP32); NP: 1 (payoff_single) or NPAY (payoff_mask);
// TRACK: keep Asian sums and running minima; F: indices per word (1 = unpacked);
// X32: the correction estimator's exact side in FP32 (FP32 inverse normal and
// FP32 Algorithm 1 arithmetic) instead of FP64.
template <int EST, int ARITH, bool MIL, int NP, bool TRACK, int F, bool X32 = false>
struct PathBody {
    static constexpr int WPB = 4 * F;                                  // normals per block
    static constexpr int WPB_TZ = 2 + (F % 2 ? 0 : (F % 4 ? 1 : (F % 8 ? 2 : 3)));   // trailing zeros
    static constexpr bool HAS_EXACT = EST != MLMC_EST_APPROX;
    static constexpr bool HAS_TABLE = EST != MLMC_EST_PLAIN;
    static constexpr bool FIXED = ARITH == MLMC_ARITH_FIXED;
    static constexpr bool PLAIN32 = EST == MLMC_EST_PLAIN && ARITH == MLMC_ARITH_FP32;
    // table entry: FP32 Euler needs only s_k; the others (Z~_k, s_k)
    static constexpr bool HALF = ARITH == MLMC_ARITH_FP16;
    // the float low-precision side's type (FP16 or FP32)
    using AT = typename std::conditional<HALF, _Float16, float>::type;
    static constexpr int TAB_BYTES = !HAS_TABLE ? 0 : (HALF ? 4 : 8);
    // the exact side in FP32: the plain-FP32 estimator, or a correction with X32
    static constexpr bool EXACT32 = PLAIN32 || (EST == MLMC_EST_CORR && X32);
    using ExactT = typename std::conditional<EXACT32, float, double>::type;

    // tab: table of 2^q entries (LDS on the device, host memory in checks)
    __host__ __device__ __forceinline__ static void run_group(const LevelDev& L, const WorkDev& W,
                                                              uint64_t g, const void* tab,
                                                              Acc<NP>& acc) {
        const int lev = L.level;
        // group = lcm(2^lev, WPB) stream positions (group_span): whole paths, whole blocks
        const uint64_t S = (uint64_t(WPB) << lev) >> (lev < WPB_TZ ? lev : WPB_TZ);
        const uint32_t nblk = static_cast<uint32_t>(S / WPB);
        const uint64_t path0 = g * (S >> lev);
        const bool coarse_on = lev >= 1;
        const int q = L.q;
        const uint32_t qmask = (1u << q) - 1u;
        uint64_t blk = g * nblk;

        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        uint32_t first_word = 0, first_index = 0;

        for (uint32_t ib = 0; ib < nblk; ++ib, ++blk) {
            u32x4 r = philox4x32_10(
                u32x4{static_cast<uint32_t>(blk), static_cast<uint32_t>(blk >> 32), W.c2, W.c3},
                W.k0, W.k1);
            if (HAS_EXACT) {
                // one word per step; a rolled loop keeps a single copy of the exact
                // inverse normal (the words rotate through r.x)
#pragma unroll 1
                for (int wi = 0; wi < 4; ++wi) {
                    const uint32_t J = r.x;
                    r.x = r.y;
                    r.y = r.z;
                    r.z = r.w;
                    step(L, W, tab, ib * 4u + wi, (wi & 1) != 0, J, 0, path0, ex, ap, ax,
                         first_word, first_index, acc);
                }
            } else {
                const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
                for (int wi = 0; wi < 4; ++wi) {
#pragma unroll
                    for (int fi = 0; fi < F; ++fi)
                        step(L, W, tab, (ib * 4u + wi) * F + fi, ((wi * F + fi) & 1) != 0, wd[wi], fi,
                             path0, ex, ap, ax, first_word, first_index, acc);
                }
            }
        }
    }

    // The word whose uniform the exact side inverts: J itself, or (Method 2) J with
    // its top q bits replaced by pi(top q bits) -- pi in the level's table entry.
    __host__ __device__ __forceinline__ static uint32_t coupled_word(const LevelDev& L, const void* tab,
                                                                     uint32_t J) {
        if (EST != MLMC_EST_CORR || !L.perm_off) return J;
        const uint16_t* pi = reinterpret_cast<const uint16_t*>(static_cast<const uint8_t*>(tab) + L.perm_off);
        const int sh = 32 - L.q;
        return (uint32_t(pi[J >> sh]) << sh) | (J & ((1u << sh) - 1u));
    }

    // Table index in field fi of a uniform word: q bits, fields from the most
    // significant end (F == 1: the top q bits).
    __host__ __device__ __forceinline__ static uint32_t index_field(uint32_t J, int fi, int q) {
        if (F == 1) return J >> (32 - q);
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_ubfe(J, static_cast<uint32_t>(32 - q * (fi + 1)), static_cast<uint32_t>(q));
#else
        return (J >> (32 - q * (fi + 1))) & ((1u << q) - 1u);
#endif
    }

    // Stream position sl of the group (odd = sl & 1, known at compile time when
    // unrolled since 4F is even); J the word holding it, fi its field.
    __host__ __device__ __forceinline__ static void step(
        const LevelDev& L, const WorkDev& W, const void* tab, uint32_t sl, bool odd, uint32_t J,
        int fi, uint64_t path0, FSide<ExactT>& ex, FSide<AT>& ap, XSide& ax,
        uint32_t& first_word, uint32_t& first_index, Acc<NP>& acc) {
        const int lev = L.level;
        const uint32_t N = 1u << lev;
        const uint32_t n = sl & (N - 1u);
        const bool coarse_on = lev >= 1;
        const int q = L.q;
        if (n == 0) {
            if (HAS_EXACT) ex.init();
            if (HAS_TABLE) { if (FIXED) ax.init(L); else ap.init(); }
        }
        uint32_t k = 0;
        if (HAS_TABLE) k = index_field(J, fi, q);
        if (n == 0) { first_word = J; first_index = k; }
        if (HAS_EXACT) {
            if (EXACT32) exact_step<MIL>(ex, norminv_f32(coupled_word(L, tab, J)), L, coarse_on, odd, TRACK);
            else exact_step<MIL>(ex, norminv_f64(coupled_word(L, tab, J)), L, coarse_on, odd, TRACK);
        }
        if (HAS_TABLE) {
            if (FIXED) {
                const int2 e = static_cast<const int2*>(tab)[k];
                fixed_step<MIL>(ax, e.x, e.y, L, coarse_on, odd, TRACK);
            } else {
                const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[k];
                table_step<MIL, AT>(ap, e.z, e.s, L, coarse_on, odd, TRACK);
            }
        }
        if (n == N - 1u) {
            const uint64_t pidx = path0 + (sl >> lev);
            if (pidx >= W.path_begin && pidx < W.path_end)
                finish(L, W, pidx, ex, ap, ax, first_word, first_index, acc);
        }
    }

    // One path of a work whose words and exact normals were computed ahead by
    // k_normals (works with few, long paths: the inverse normal then leaves the
    // path's sequential chain).  Same steps and records as run_group.
    // Steps 0 .. N-1 of one buffered path, AH (<= N, dividing N) loads in flight.
    // Loads are unconditional (the index is clamped to the last step) so that no
    // branch join forces an early wait on them.
    template <uint32_t AH>
    __host__ __device__ __forceinline__ static void buffered_steps(
        const LevelDev& L, uint32_t N, uint64_t P, uint64_t col, const MLMC_GLOBAL uint32_t* Jb,
        const MLMC_GLOBAL ExactT* Zb, const void* tab, FSide<ExactT>& ex, FSide<AT>& ap, XSide& ax) {
        const int q = L.q;
        uint32_t jq[AH];
        ExactT zq[AH];
#pragma unroll
        for (uint32_t h = 0; h < AH; ++h) {
            jq[h] = Jb[uint64_t(h) * P + col];
            zq[h] = Zb[uint64_t(h) * P + col];
        }
        for (uint32_t n = 0; n < N; n += AH) {
#pragma unroll
            for (uint32_t h = 0; h < AH; ++h) {
                const uint32_t J = jq[h];
                const ExactT Z = zq[h];
                const uint32_t nn = n + AH + h < N ? n + AH + h : N - 1u;
                jq[h] = Jb[uint64_t(nn) * P + col];
                zq[h] = Zb[uint64_t(nn) * P + col];
                exact_step<MIL>(ex, Z, L, true, (h & 1u) == 1u, TRACK);
                if (HAS_TABLE) {
                    const uint32_t k = J >> (32 - q);
                    if (FIXED) {
                        const int2 e = static_cast<const int2*>(tab)[k];
                        fixed_step<MIL>(ax, e.x, e.y, L, true, (h & 1u) == 1u, TRACK);
                    } else {
                        const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[k];
                        table_step<MIL, AT>(ap, e.z, e.s, L, true, (h & 1u) == 1u, TRACK);
                    }
                }
            }
        }
    }

    __host__ __device__ __forceinline__ static void run_path_buffered(const LevelDev& L,
                                                                      const WorkDev& W,
                                                                      uint64_t pidx, const void* tab,
                                                                      Acc<NP>& acc) {
        const int lev = L.level;
        const uint32_t N = 1u << lev;
        const uint64_t P = W.path_end - W.path_begin;
        const uint64_t col = pidx - W.path_begin;
        const MLMC_GLOBAL ExactT* Zb = global_ptr<const ExactT>(W.zbuf);
        const MLMC_GLOBAL uint32_t* Jb = global_ptr<const uint32_t>(W.jbuf);
        const int q = L.q;
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        ex.init();
        if (HAS_TABLE) { if (FIXED) ax.init(L); else ap.init(); }
        const uint32_t first_word = Jb[col];
        const uint32_t first_index = HAS_TABLE ? (first_word >> (32 - q)) : 0u;
        // The step loop is a serial chain: the word and normal of step n + AH are
        // loaded while step n computes, so a global load's latency is paid once per AH
        // steps.  N >= 4 is a power of two (steps come in (even, odd) pairs).
        if (N >= 8) buffered_steps<8>(L, N, P, col, Jb, Zb, tab, ex, ap, ax);
        else buffered_steps<4>(L, N, P, col, Jb, Zb, tab, ex, ap, ax);
        finish(L, W, pidx, ex, ap, ax, first_word, first_index, acc);
    }

    // The estimator's sample for payoff p from the final path states: Ye (exact side
    // dP), Ya (approximate side dP~, FP64 view), Yint (fixed point: dP~ as an
    // integer), Y (the estimator's sample).
    __host__ __device__ __forceinline__ static void sample(const LevelDev& L, int p,
                                                           const FSide<ExactT>& ex,
                                                           const FSide<AT>& ap, XSide& ax,
                                                           ExactT ek, ExactT eb, double& Ye,
                                                           double& Ya, int64_t& Yint, double& Y) {
        const int lev = L.level;
        Ye = 0.0;
        Ya = 0.0;
        Yint = 0;
        if (HAS_EXACT) {
            const ExactT pf = ex.payoff(p, true, lev, ek, eb);
            const ExactT pc = lev ? ex.payoff(p, false, lev - 1, ek, eb) : ExactT(0);
            Ye = static_cast<double>(pf - pc);
        }
        if (HAS_TABLE) {
            if (FIXED) {
                const int64_t pf = ax.payoff(p, true, lev, L);
                const int64_t pc = lev ? ax.payoff(p, false, lev - 1, L) : 0;
                Yint = pf - pc;
                Ya = ldexp(static_cast<double>(Yint), -L.fX);
            } else {
#pragma clang fp contract(off)
                const LpConst<AT> c = lp_const<AT>(L);
                const AT pf = ap.payoff(p, true, lev, c.k, c.b);
                const AT pc = lev ? ap.payoff(p, false, lev - 1, c.k, c.b) : AT(0);
                const AT y = pf - pc;
                Ya = static_cast<double>(y);
            }
        }
        if (EST == MLMC_EST_PLAIN) Y = Ye;
        else if (EST == MLMC_EST_APPROX) Y = Ya;
        else Y = Ye - Ya;
    }

    // ---- level 0 of the approximate estimator as an index histogram.  A level-0
    // path has one step, so with Method-1 normals its sample is a function of its
    // table index k alone: sum_paths f(Y) = sum_k c_k f(Y(k)).  The kernel counts
    // the indices of a tile and evaluates Y(k) once per index with the path code.
    static constexpr bool HIST = EST == MLMC_EST_APPROX;

    // the level-0 path of index k (its final states)
    __host__ __device__ __forceinline__ static void level0_path(const LevelDev& L, const void* tab,
                                                                uint32_t k, FSide<AT>& ap,
                                                                XSide& ax) {
        if (FIXED) {
            ax.init(L);
            const int2 e = static_cast<const int2*>(tab)[k];
            fixed_step<MIL>(ax, e.x, e.y, L, false, false, TRACK);
        } else {
            ap.init();
            const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[k];
            table_step<MIL, AT>(ap, e.z, e.s, L, false, false, TRACK);
        }
    }

    // Counts the indices of level-0 group g (WPB whole paths, one Philox block),
    // calling count(k) per path in range; with a debug buffer, also writes each
    // path's record from the per-path code.
    template <class Count>
    __host__ __device__ __forceinline__ static void hist_group(const LevelDev& L, const WorkDev& W,
                                                               uint64_t g, const void* tab,
                                                               Count& count) {
        const uint64_t path0 = g * WPB;
        const u32x4 r = philox4x32_10(
            u32x4{static_cast<uint32_t>(g), static_cast<uint32_t>(g >> 32), W.c2, W.c3}, W.k0, W.k1);
        const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
        const bool full = path0 >= W.path_begin && path0 + WPB <= W.path_end;
        const int q = L.q;
        if (full && !W.debug) {
            // every path of the group is in range and no records: count only
#pragma unroll
            for (int wi = 0; wi < 4; ++wi)
#pragma unroll
                for (int fi = 0; fi < F; ++fi) count(index_field(wd[wi], fi, q));
            return;
        }
#pragma unroll
        for (int wi = 0; wi < 4; ++wi) {
#pragma unroll
            for (int fi = 0; fi < F; ++fi) {
                const uint32_t J = wd[wi];
                const uint32_t k = index_field(J, fi, q);
                const uint64_t pidx = path0 + uint64_t(wi * F + fi);
                if (full || (pidx >= W.path_begin && pidx < W.path_end)) {
                    count(k);
                    if (W.debug) {
                        FSide<ExactT> ex;
                        FSide<AT> ap;
                        XSide ax;
                        level0_path(L, tab, k, ap, ax);
                        Acc<NP> scratch;
                        acc_zero(scratch);
                        finish(L, W, pidx, ex, ap, ax, J, k, scratch);
                    }
                }
            }
        }
    }

    // ---- level 0 of the FP32 approximate estimator from a table of per-index
    // samples: Y(k) is computed once per level (ysample) into LDS and every path adds
    // its own sample (the same values as the per-path code; per group in four
    // interleaved partial sums), with one table read per path instead of the path
    // arithmetic.
    // (Fixed point keeps the index histogram: its exact integer sums per path would
    // cost more than a count.)
    static constexpr bool YTAB = HIST && !FIXED;

    // The level-0 sample of index k for each payoff slot (the FP32 payoff
    // difference, held in FP64 so that no path converts it), written to
    // ytab[slot * entries + k]; returns false if one is not finite (the caller then
    // counts instead).
    __host__ __device__ __forceinline__ static bool ysample(const LevelDev& L, const void* tab,
                                                            uint32_t k, double* ytab) {
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        level0_path(L, tab, k, ap, ax);
        bool ok = true;
#pragma unroll
        for (int slot = 0; slot < NP; ++slot) {
            const int p = NP == 1 ? L.payoff_single : slot;
            double y = 0.0;
            if (NP == 1 || ((L.payoff_mask >> p) & 1u)) {
                double Ye, Ya, Y;
                int64_t Yint;
                sample(L, p, ex, ap, ax, ExactT(0), ExactT(0), Ye, Ya, Yint, Y);
                ok = ok && __builtin_isfinite(Y);
                y = static_cast<double>(static_cast<float>(Y));
            }
            ytab[slot * L.table_entries + k] = y;
        }
        return ok;
    }

    // Adds the level-0 samples of group g (WPB paths, one Philox block) from the
    // per-index table; partial groups and debug records take the checked loop.
    __host__ __device__ __forceinline__ static void ytab_group(const LevelDev& L, const WorkDev& W,
                                                               uint64_t g, const void* tab,
                                                               const double* ytab, Acc<NP>& acc) {
        const uint64_t path0 = g * WPB;
        const u32x4 r = philox4x32_10(
            u32x4{static_cast<uint32_t>(g), static_cast<uint32_t>(g >> 32), W.c2, W.c3}, W.k0, W.k1);
        const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
        const bool full = path0 >= W.path_begin && path0 + WPB <= W.path_end;
        const int q = L.q;
        const uint32_t E = L.table_entries;
        // path j of the group adds to partial sum j mod 4 and the partials join the
        // accumulator as (p0 + p1) + (p2 + p3): four short dependent FP64 chains
        // instead of one of length 4F, in the same order in both branches
        double p1[4][NP], p2[4][NP];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int slot = 0; slot < NP; ++slot) p1[c][slot] = p2[c][slot] = 0.0;
        if (full && !W.debug) {
#pragma unroll
            for (int wi = 0; wi < 4; ++wi)
#pragma unroll
                for (int fi = 0; fi < F; ++fi) {
                    const uint32_t k = index_field(wd[wi], fi, q);
                    const int c = (wi * F + fi) & 3;
#pragma unroll
                    for (int slot = 0; slot < NP; ++slot) {
                        const double Y = ytab[slot * E + k];
                        p1[c][slot] += Y;
                        p2[c][slot] = fma(Y, Y, p2[c][slot]);
                    }
                }
            acc.n += WPB;
        } else {
#pragma unroll
            for (int wi = 0; wi < 4; ++wi) {
#pragma unroll
                for (int fi = 0; fi < F; ++fi) {
                    const uint32_t J = wd[wi];
                    const uint32_t k = index_field(J, fi, q);
                    const uint64_t pidx = path0 + uint64_t(wi * F + fi);
                    const int c = (wi * F + fi) & 3;
                    if (full || (pidx >= W.path_begin && pidx < W.path_end)) {
                        if (W.debug) {
                            FSide<ExactT> ex;
                            FSide<AT> ap;
                            XSide ax;
                            level0_path(L, tab, k, ap, ax);
                            Acc<NP> scratch;
                            acc_zero(scratch);
                            finish(L, W, pidx, ex, ap, ax, J, k, scratch);
                        }
#pragma unroll
                        for (int slot = 0; slot < NP; ++slot) {
                            const double Y = ytab[slot * E + k];
                            p1[c][slot] += Y;
                            p2[c][slot] = fma(Y, Y, p2[c][slot]);
                        }
                        acc.n += 1;
                    }
                }
            }
        }
#pragma unroll
        for (int slot = 0; slot < NP; ++slot) {
            acc.s1[slot] += (p1[0][slot] + p1[1][slot]) + (p1[2][slot] + p1[3][slot]);
            acc.s2[slot] += (p2[0][slot] + p2[1][slot]) + (p2[2][slot] + p2[3][slot]);
        }
    }

    // Adds c copies of the level-0 sample of index k to acc.
    __host__ __device__ __forceinline__ static void hist_accumulate(const LevelDev& L,
                                                                    const void* tab, uint32_t k,
                                                                    uint32_t c, Acc<NP>& acc) {
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        level0_path(L, tab, k, ap, ax);
        const double cd = static_cast<double>(c);
#pragma unroll
        for (int slot = 0; slot < NP; ++slot) {
            const int p = NP == 1 ? L.payoff_single : slot;
            if (NP != 1 && !((L.payoff_mask >> p) & 1u)) continue;
            double Ye, Ya, Y;
            int64_t Yint;
            sample(L, p, ex, ap, ax, ExactT(0), ExactT(0), Ye, Ya, Yint, Y);
            if (!__builtin_isfinite(Y)) { acc.nonfinite += c; continue; }
            acc.s1[slot] = fma(cd, Y, acc.s1[slot]);            // c Y is exact
            acc.s2[slot] = fma(cd * Y, Y, acc.s2[slot]);
            if (FIXED) {
                acc.i1[slot] += static_cast<int64_t>(c) * Yint;
                const uint64_t a = static_cast<uint64_t>(Yint < 0 ? -Yint : Yint);
                const uint64_t sq = a * a;
#if defined(__HIP_DEVICE_COMPILE__)
                const uint64_t hi = __umul64hi(sq, uint64_t(c));
#else
                const uint64_t hi = static_cast<uint64_t>((static_cast<unsigned __int128>(sq) * c) >> 64);
#endif
                const uint64_t lo = sq * uint64_t(c);
                const uint64_t nlo = acc.i2lo[slot] + lo;
                acc.i2hi[slot] += hi + (nlo < lo ? 1u : 0u);
                acc.i2lo[slot] = nlo;
            }
        }
        acc.n += c;
        if (FIXED) acc.sat += c * ax.nsat;
    }

    // ---- the approximate estimator above level 0: whole groups without a debug
    // buffer.  Where a path starts and ends within the group is fixed by the level, so
    // this loop places the initialisations and the final samples by construction
    // instead of testing each step as the general code does (there the per-step tests
    // become selects on every state variable).  The steps (table_step, fixed_step),
    // samples (finish) and their order are the general code's, so the sums are the
    // same bit for bit.  Power-of-two blocks of 4F positions only.
    static constexpr bool FASTG = EST == MLMC_EST_APPROX && (WPB & (WPB - 1)) == 0;

    // one table step of the approximate side at stream position j of a block
    __host__ __device__ __forceinline__ static void approx_step(const LevelDev& L, const void* tab, uint32_t k,
                                                                bool odd, FSide<AT>& ap, XSide& ax) {
        if constexpr (FIXED) {
            const int2 e = static_cast<const int2*>(tab)[k];
            fixed_step<MIL>(ax, e.x, e.y, L, true, odd, TRACK);
        } else {
            const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[k];
            table_step<MIL, AT>(ap, e.z, e.s, L, true, odd, TRACK);
        }
    }
    __host__ __device__ __forceinline__ static void approx_init(const LevelDev& L, FSide<AT>& ap, XSide& ax) {
        if constexpr (FIXED) ax.init(L);
        else ap.init();
    }

    // the 4F table indices of Philox block b, position by position
    __host__ __device__ __forceinline__ static void block_indices(const WorkDev& W, uint64_t b, int q,
                                                                  uint32_t (&k)[WPB]) {
        const u32x4 r = philox4x32_10(
            u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), W.c2, W.c3}, W.k0, W.k1);
        const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < WPB; ++j) k[j] = index_field(wd[j / F], j % F, q);
    }

    // levels with 2^LEV < 4F steps: block g holds 4F / 2^LEV whole paths
    template <int LEV>
    __host__ __device__ __forceinline__ static void short_paths(const LevelDev& L, const WorkDev& W,
                                                                uint64_t g, const void* tab, Acc<NP>& acc) {
        constexpr int N = 1 << LEV;
        uint32_t k[WPB];
        block_indices(W, g, L.q, k);
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
#pragma unroll
        for (int j = 0; j < WPB; ++j) {
            if ((j & (N - 1)) == 0) approx_init(L, ap, ax);
            approx_step(L, tab, k[j], (j & 1) != 0, ap, ax);
            if ((j & (N - 1)) == N - 1) finish(L, W, 0, ex, ap, ax, 0u, 0u, acc);
        }
    }

    // levels with 2^level >= 4F steps: group g is path g, over 2^level / 4F blocks
    __host__ __device__ __forceinline__ static void long_path(const LevelDev& L, const WorkDev& W,
                                                              uint64_t g, const void* tab, Acc<NP>& acc) {
        const uint32_t nblk = (1u << L.level) / WPB;
        uint64_t b = g * nblk;
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        approx_init(L, ap, ax);
        for (uint32_t ib = 0; ib < nblk; ++ib, ++b) {
            uint32_t k[WPB];
            block_indices(W, b, L.q, k);
#pragma unroll
            for (int j = 0; j < WPB; ++j) approx_step(L, tab, k[j], (j & 1) != 0, ap, ax);
        }
        finish(L, W, 0, ex, ap, ax, 0u, 0u, acc);
    }

    // ---- FP16, two paths per lane: a thread's next two whole groups ga < gb above
    // level 0 (no records, no path functionals) advance together, each operation of
    // the two paths' chains one packed instruction (v_pk_mul_f16 / v_pk_add_f16,
    // rounded per element as the scalar operation), and finish in the order ga, gb:
    // the per-path values and the order of accumulation of run_group_fast on ga, then
    // on gb.
    static constexpr bool PAIR = FASTG && HALF && !TRACK;

    __device__ __forceinline__ static void run_group_pair(const LevelDev& L, const WorkDev& W, uint64_t ga,
                                                          uint64_t gb, const void* tab, Acc<NP>& acc) {
        if constexpr (PAIR) {
            // long paths (a group is one path), both in the work's range
            if (L.level >= WPB_TZ && !W.debug && ga >= W.path_begin && gb < W.path_end) {
                long_path_pair(L, W, ga, gb, tab, acc);
                return;
            }
        }
        run_group_fast(L, W, ga, tab, acc);
        run_group_fast(L, W, gb, tab, acc);
    }

    __device__ __forceinline__ static void long_path_pair(const LevelDev& L, const WorkDev& W, uint64_t ga,
                                                          uint64_t gb, const void* tab, Acc<NP>& acc) {
#pragma clang fp contract(off)
        const uint32_t nblk = (1u << L.level) / WPB;
        const LpConst<_Float16> c = lp_const<_Float16>(L);
        const half2v con1c = {c.con1c, c.con1c}, con2 = {c.con2, c.con2}, con3 = {c.con3, c.con3};
        const half2v two = {_Float16(2), _Float16(2)};
        const TabPair<_Float16>* T = static_cast<const TabPair<_Float16>*>(tab);
        half2v xf = {_Float16(1), _Float16(1)}, xc = xf, zp = {_Float16(0), _Float16(0)};
        uint64_t ba = ga * nblk, bb = gb * nblk;
        for (uint32_t ib = 0; ib < nblk; ++ib, ++ba, ++bb) {
            uint32_t ka[WPB], kb[WPB];
            block_indices(W, ba, L.q, ka);
            block_indices(W, bb, L.q, kb);
#pragma unroll
            for (int j = 0; j < WPB; ++j) {
                const TabPair<_Float16> ea = T[ka[j]], eb = T[kb[j]];
                const half2v z = {ea.z, eb.z}, sk = {ea.s, eb.s};
                const half2v mul2 = xf * sk;                    // fine: x + x s_k
                xf = xf + mul2;
                if ((j & 1) == 0) {
                    zp = z;
                } else {                                        // coarse: x + x m(zp + z)
                    const half2v zs = zp + z;
                    const half2v mul1 = con2 * zs;
                    half2v m = con1c + mul1;
                    if (MIL) {
                        const half2v zsq = zs * zs;
                        const half2v zm1 = zsq - two;
                        const half2v mul3 = con3 * zm1;
                        m = m + mul3;
                    }
                    const half2v mc = xc * m;
                    xc = xc + mc;
                }
            }
        }
        FSide<ExactT> ex;
        XSide ax;
        FSide<_Float16> a, b;
        a.init();
        b.init();
        a.xf = xf.x;
        a.xc = xc.x;
        b.xf = xf.y;
        b.xc = xc.y;
        finish(L, W, 0, ex, a, ax, 0u, 0u, acc);
        finish(L, W, 0, ex, b, ax, 0u, 0u, acc);
    }

    // Philox block b of W's stream for the exact-normal loops.  The keys are marked
    // as rewritten here, so their 20 round keys are formed per call by scalar adds
    // instead of being hoisted out of the loop, where beside the FP64 inverse
    // normal's coefficients they outgrow the scalar registers and end up in
    // vector-register lanes (a v_readlane and a wait state per round).
    __host__ __device__ __forceinline__ static u32x4 philox_group_keys(const WorkDev& W, uint64_t b) {
        uint32_t k0 = W.k0, k1 = W.k1;
#if defined(__HIP_DEVICE_COMPILE__)
        asm volatile("" : "+s"(k0), "+s"(k1));
#endif
        return philox4x32_10(u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), W.c2, W.c3}, k0, k1);
    }

    // The same loop for the exact-normal estimators (plain; correction with a float
    // table side), one word per step (F = 1): steps come in (even, odd) pairs, and the
    // pairs run in a rolled loop so that one copy of the inverse normal serves each
    // parity.
    static constexpr bool EXG = HAS_EXACT && !FIXED && F == 1;

    // the (even, odd) step pair of words (J0, J1): exact side, then the table side
    __host__ __device__ __forceinline__ static void exact_pair(const LevelDev& L, const void* tab, uint32_t J0,
                                                               uint32_t J1, FSide<ExactT>& ex, FSide<AT>& ap) {
        const int sh = 32 - L.q;
        if (EXACT32) exact_step<MIL>(ex, norminv_f32(coupled_word(L, tab, J0)), L, true, false, TRACK);
        else exact_step<MIL>(ex, norminv_f64(coupled_word(L, tab, J0)), L, true, false, TRACK);
        if (HAS_TABLE) {
            const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[J0 >> sh];
            table_step<MIL, AT>(ap, e.z, e.s, L, true, false, TRACK);
        }
        if (EXACT32) exact_step<MIL>(ex, norminv_f32(coupled_word(L, tab, J1)), L, true, true, TRACK);
        else exact_step<MIL>(ex, norminv_f64(coupled_word(L, tab, J1)), L, true, true, TRACK);
        if (HAS_TABLE) {
            const TabPair<AT> e = static_cast<const TabPair<AT>*>(tab)[J1 >> sh];
            table_step<MIL, AT>(ap, e.z, e.s, L, true, true, TRACK);
        }
    }

    __host__ __device__ __forceinline__ static void exact_group_fast(const LevelDev& L, const WorkDev& W,
                                                                     uint64_t g, const void* tab,
                                                                     Acc<NP>& acc) {
        FSide<ExactT> ex;
        FSide<AT> ap;
        XSide ax;
        if (L.level == 1) {
            // block g holds paths 2g and 2g + 1, two steps each
            u32x4 r = philox_group_keys(W, g);
#pragma unroll 1
            for (int p = 0; p < 2; ++p) {
                const uint32_t J0 = r.x, J1 = r.y;
                r.x = r.z;
                r.y = r.w;
                ex.init();
                if (HAS_TABLE) ap.init();
                exact_pair(L, tab, J0, J1, ex, ap);
                finish(L, W, 0, ex, ap, ax, 0u, 0u, acc);
            }
            return;
        }
        // level >= 2: path g over 2^level / 4 blocks, two pairs per block
        const uint32_t nblk = (1u << L.level) / 4u;
        uint64_t b = g * nblk;
        ex.init();
        if (HAS_TABLE) ap.init();
        for (uint32_t ib = 0; ib < nblk; ++ib, ++b) {
            u32x4 r = philox_group_keys(W, b);
#pragma unroll 1
            for (int p = 0; p < 2; ++p) {
                const uint32_t J0 = r.x, J1 = r.y;
                r.x = r.z;
                r.y = r.w;
                exact_pair(L, tab, J0, J1, ex, ap);
            }
        }
        finish(L, W, 0, ex, ap, ax, 0u, 0u, acc);
    }

    // group g of a level >= 1 work: these loops when the group is whole and there is no
    // debug buffer, else the general code
    __host__ __device__ __forceinline__ static void run_group_fast(const LevelDev& L, const WorkDev& W,
                                                                   uint64_t g, const void* tab,
                                                                   Acc<NP>& acc) {
        const int lev = L.level;
        const uint64_t paths = lev < WPB_TZ ? uint64_t(WPB) >> lev : 1u;
        const uint64_t path0 = g * paths;
        if (lev == 0 || W.debug || path0 < W.path_begin || path0 + paths > W.path_end) {
            run_group(L, W, g, tab, acc);
            return;
        }
        if constexpr (EXG) {
            exact_group_fast(L, W, g, tab, acc);
        } else {
            switch (lev) {
                case 1: if constexpr (WPB_TZ > 1) { short_paths<1>(L, W, g, tab, acc); return; } break;
                case 2: if constexpr (WPB_TZ > 2) { short_paths<2>(L, W, g, tab, acc); return; } break;
                case 3: if constexpr (WPB_TZ > 3) { short_paths<3>(L, W, g, tab, acc); return; } break;
                case 4: if constexpr (WPB_TZ > 4) { short_paths<4>(L, W, g, tab, acc); return; } break;
                default: break;
            }
            long_path(L, W, g, tab, acc);
        }
    }

    // ---- level 0 of the exact-normal estimators (plain; correction with a float
    // table side), without a debug buffer.  A level-0 path is one step, so the loop is
    // written for it (no step counting or coarse bookkeeping), and the correction
    // estimator's approximate-side sample Ya -- a function of the path's table index
    // alone -- comes from a per-index table built once per level (ya_sample), as the
    // approximate estimator's level 0 does.  Each path's operations and the order in
    // which they join the accumulator are those of run_group and finish, so the sums
    // are the same bit for bit.
    static constexpr bool EX0 = HAS_EXACT && !FIXED && F == 1;

    // Ya(k) of each payoff slot (the FP64 view that sample() forms), written to
    // yat[slot * entries + k]
    __host__ __device__ __forceinline__ static void ya_sample(const LevelDev& L, const void* tab,
                                                              uint32_t k, double* yat) {
        FSide<ExactT> ex;
        ex.init();
        FSide<AT> ap;
        XSide ax;
        level0_path(L, tab, k, ap, ax);
#pragma unroll
        for (int slot = 0; slot < NP; ++slot) {
            const int p = NP == 1 ? L.payoff_single : slot;
            double y = 0.0;
            if (NP == 1 || ((L.payoff_mask >> p) & 1u)) {
                double Ye, Ya, Y;
                int64_t Yint;
                sample(L, p, ex, ap, ax, ExactT(L.k), ExactT(L.b), Ye, Ya, Yint, Y);
                y = Ya;
            }
            yat[slot * L.table_entries + k] = y;
        }
    }

    // The four level-0 paths 4g .. 4g + 3 of group g (one Philox block, one word per
    // path); yat: the level's Ya table (correction estimator only).
    __host__ __device__ __forceinline__ static void exact0_group(const LevelDev& L, const WorkDev& W,
                                                                 uint64_t g, const void* tab,
                                                                 const double* yat, Acc<NP>& acc) {
        const u32x4 r = philox_group_keys(W, g);
        const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
        const uint64_t path0 = g * 4u;
        const ExactT ek = EXACT32 ? ExactT(L.fk) : ExactT(L.k);
        const ExactT eb = EXACT32 ? ExactT(L.fb) : ExactT(L.b);
        const int sh = 32 - L.q;
        // the four inverse normals together (norminv_*_x4: interleaved chains, the
        // rare tails after), the same values as one at a time
        ExactT Z[4];
        uint32_t Je[4];
#pragma unroll
        for (int wi = 0; wi < 4; ++wi) Je[wi] = coupled_word(L, tab, wd[wi]);
        if constexpr (EXACT32) norminv_f32_x4(Je, Z);
        else norminv_f64_x4(Je, Z);
#pragma unroll
        for (int wi = 0; wi < 4; ++wi) {
            const uint32_t J = wd[wi];
            FSide<ExactT> ex;
            ex.init();
            exact_step<MIL>(ex, Z[wi], L, false, false, TRACK);
            const uint64_t pidx = path0 + static_cast<uint32_t>(wi);
            if (pidx < W.path_begin || pidx >= W.path_end) continue;
            const uint32_t k = HAS_TABLE ? (J >> sh) : 0u;
#pragma unroll
            for (int slot = 0; slot < NP; ++slot) {
                const int p = NP == 1 ? L.payoff_single : slot;
                if (NP != 1 && !((L.payoff_mask >> p) & 1u)) continue;
                const ExactT pf = ex.payoff(p, true, 0, ek, eb);
                const double Ye = static_cast<double>(pf - ExactT(0));
                double Y = Ye;
                if (EST == MLMC_EST_CORR) Y = Ye - yat[slot * L.table_entries + k];
                if (!__builtin_isfinite(Y)) { acc.nonfinite += 1; Y = 0.0; }
                acc.s1[slot] += Y;
                acc.s2[slot] = fma(Y, Y, acc.s2[slot]);
                if (EST == MLMC_EST_CORR) {
                    acc.e1[slot] += Ye;
                    acc.e2[slot] = fma(Ye, Ye, acc.e2[slot]);
                }
            }
            acc.n += 1;
        }
    }

    __host__ __device__ __forceinline__ static void finish(const LevelDev& L, const WorkDev& W,
                                                           uint64_t pidx, const FSide<ExactT>& ex,
                                                           const FSide<AT>& ap, XSide& ax,
                                                           uint32_t first_word,
                                                           uint32_t first_index, Acc<NP>& acc) {
        const int lev = L.level;
        MLMC_GLOBAL mlmc_path_record* rec =
            W.debug ? global_ptr<mlmc_path_record>(W.debug) + (pidx - W.path_begin) : nullptr;
        const ExactT ek = EXACT32 ? ExactT(L.fk) : ExactT(L.k);
        const ExactT eb = EXACT32 ? ExactT(L.fb) : ExactT(L.b);
#pragma unroll
        for (int slot = 0; slot < NP; ++slot) {
            const int p = NP == 1 ? L.payoff_single : slot;
            if (NP != 1 && !((L.payoff_mask >> p) & 1u)) continue;
            double Ye, Ya, Y;
            int64_t Yint;
            sample(L, p, ex, ap, ax, ek, eb, Ye, Ya, Yint, Y);
            if (!__builtin_isfinite(Y)) { acc.nonfinite += 1; Y = 0.0; }
            acc.s1[slot] += Y;
            acc.s2[slot] = fma(Y, Y, acc.s2[slot]);
            if (EST == MLMC_EST_CORR) {
                acc.e1[slot] += Ye;
                acc.e2[slot] = fma(Ye, Ye, acc.e2[slot]);
            }
            if (FIXED && EST == MLMC_EST_APPROX) {
                acc.i1[slot] += Yint;
                const uint64_t a = static_cast<uint64_t>(Yint < 0 ? -Yint : Yint);
                const uint64_t sq = a * a;                       // |Y| < 2^32 by validation
                const uint64_t lo = acc.i2lo[slot] + sq;
                acc.i2hi[slot] += (lo < sq) ? 1u : 0u;
                acc.i2lo[slot] = lo;
            }
            if (rec) {
                rec->Y[p] = Y;
                if (FIXED) {
                    rec->Yraw[p] = Yint;
                } else {
                    union { double d; int64_t i; } u;
                    u.d = Ya;
                    rec->Yraw[p] = u.i;
                }
            }
        }
        acc.n += 1;
        if (FIXED) acc.sat += ax.nsat;
        if (rec) {
            rec->XN_exact = HAS_EXACT ? static_cast<double>(ex.xf) : 0.0;
            rec->XcN_exact = HAS_EXACT ? static_cast<double>(ex.xc) : 0.0;
            if (FIXED) {
                rec->XN_raw = ax.xf;
                rec->XcN_raw = ax.xc;
                rec->XN_approx = ldexp(static_cast<double>(ax.xf), -L.fX);
                rec->XcN_approx = ldexp(static_cast<double>(ax.xc), -L.fX);
            } else {
                rec->XN_raw = rec->XcN_raw = 0;
                rec->XN_approx = HAS_TABLE ? static_cast<double>(ap.xf) : 0.0;
                rec->XcN_approx = HAS_TABLE ? static_cast<double>(ap.xc) : 0.0;
            }
            rec->first_word = first_word;
            rec->first_index = first_index;
            rec->saturations = FIXED ? ax.nsat : 0u;
            rec->reserved = 0u;
        }
    }
};

}  // namespace mlmc
