// Block-level sums of the path kernels' per-thread accumulators in a fixed order
// (butterfly within each 64-lane wave, then the waves in index order), and the
// fixed-order reduction of a work's tile slots (shared by the flight reduction and
// the device sweep engine).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../common.hpp"
#include "paths.hpp"

namespace mlmc {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void wave_sum128(uint64_t& lo, uint64_t& hi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t olo = __shfl_xor(lo, o);
        const uint64_t ohi = __shfl_xor(hi, o);
        const uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1u : 0u);
        lo = nlo;
    }
}

constexpr int MAX_WAVES = 16;

struct RedLds {
    double d[MAX_WAVES][4 * NPAY];
    int64_t i1[MAX_WAVES][NPAY];
    uint64_t lo[MAX_WAVES][NPAY], hi[MAX_WAVES][NPAY];
    uint64_t c[MAX_WAVES][3];
};

// Block sum of the per-thread accumulators (butterfly in each wave, then the waves
// in index order) written by thread 0 to *out; the counts come as 64-bit values.
// FULL: the whole SlotDev (zeros in the fields the variant does not fill: a work's
// result); else only the fields the reduction reads (a tile's partial sums).
template <int NP, bool CORR, bool INTS, bool FULL>
__device__ __forceinline__ void block_store_counts(Acc<NP>& a, uint64_t cn, uint64_t csat, uint64_t cnf,
                                                   SlotDev* out, RedLds& r) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    double d[4 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        d[p] = wave_sum(a.s1[p]);
        d[NP + p] = wave_sum(a.s2[p]);
        d[2 * NP + p] = CORR ? wave_sum(a.e1[p]) : 0.0;
        d[3 * NP + p] = CORR ? wave_sum(a.e2[p]) : 0.0;
        if (INTS) {
            a.i1[p] = wave_sum(a.i1[p]);
            wave_sum128(a.i2lo[p], a.i2hi[p]);
        }
    }
    const int64_t n = wave_sum(static_cast<int64_t>(cn));
    const int64_t sat = wave_sum(static_cast<int64_t>(csat));
    const int64_t nf = wave_sum(static_cast<int64_t>(cnf));
    __syncthreads();                           // previous tile's readers are done
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 4 * NP; ++i) r.d[wave][i] = d[i];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            r.i1[wave][p] = INTS ? a.i1[p] : 0;
            r.lo[wave][p] = INTS ? a.i2lo[p] : 0;
            r.hi[wave][p] = INTS ? a.i2hi[p] : 0;
        }
        r.c[wave][0] = n;
        r.c[wave][1] = sat;
        r.c[wave][2] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        SlotDev s;
        for (int p = 0; p < NPAY; ++p) {
            s.s1[p] = s.s2[p] = s.e1[p] = s.e2[p] = 0.0;
            s.i1[p] = 0;
            s.i2lo[p] = s.i2hi[p] = 0;
        }
        s.n = s.sat = s.nonfinite = s.pad = 0;
        for (int w = 0; w < nw; ++w) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                s.s1[p] += r.d[w][p];
                s.s2[p] += r.d[w][NP + p];
                s.e1[p] += r.d[w][2 * NP + p];
                s.e2[p] += r.d[w][3 * NP + p];
                s.i1[p] += r.i1[w][p];
                const uint64_t nlo = s.i2lo[p] + r.lo[w][p];
                s.i2hi[p] += r.hi[w][p] + (nlo < s.i2lo[p] ? 1u : 0u);
                s.i2lo[p] = nlo;
            }
            s.n += r.c[w][0];
            s.sat += r.c[w][1];
            s.nonfinite += r.c[w][2];
        }
        if (FULL) {
            *out = s;
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                out->s1[p] = s.s1[p];
                out->s2[p] = s.s2[p];
                if (CORR) {
                    out->e1[p] = s.e1[p];
                    out->e2[p] = s.e2[p];
                }
                if (INTS) {
                    out->i1[p] = s.i1[p];
                    out->i2lo[p] = s.i2lo[p];
                    out->i2hi[p] = s.i2hi[p];
                }
            }
            out->n = s.n;
            out->sat = s.sat;
            out->nonfinite = s.nonfinite;
        }
    }
}

// a tile's partial sums
template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void block_store(Acc<NP>& a, SlotDev* out, RedLds& r) {
    block_store_counts<NP, CORR, INTS, false>(a, a.n, a.sat, a.nonfinite, out, r);
}

// Sums of one work item's tile slots in a fixed order that depends only on the
// number of slots: lane v of wave w (8 waves) adds slots 64 c + v for chunks
// c = w, w + 8, w + 16, ... in order; a butterfly adds each wave's lanes and the
// waves are added in index order.  Only the payoffs, correction sums and integer
// sums of the work's kernel variant are added; the rest of the result is zero.
constexpr int REDUCE_THREADS = 512;
constexpr int REDUCE_WAVES = REDUCE_THREADS / 64;

template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void reduce_work(const SlotDev* __restrict__ sl, uint32_t ns,
                                            SlotDev* __restrict__ dst, RedLds& r) {
    Acc<NP> a;
    acc_zero(a);
    uint64_t n = 0, sat = 0, nf = 0;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll 4
    for (uint32_t i = wave * 64u + lane; i < ns; i += REDUCE_THREADS) {
        const SlotDev& x = sl[i];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            a.s1[p] += x.s1[p];
            a.s2[p] += x.s2[p];
            if (CORR) {
                a.e1[p] += x.e1[p];
                a.e2[p] += x.e2[p];
            }
            if (INTS) {
                a.i1[p] += x.i1[p];
                const uint64_t lo = a.i2lo[p] + x.i2lo[p];
                a.i2hi[p] += x.i2hi[p] + (lo < a.i2lo[p] ? 1u : 0u);
                a.i2lo[p] = lo;
            }
        }
        n += x.n;
        sat += x.sat;
        nf += x.nonfinite;
    }
    block_store_counts<NP, CORR, INTS, true>(a, n, sat, nf, dst, r);
}

}  // namespace mlmc
