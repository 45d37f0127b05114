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

// Wave sums (butterfly) of one wave's accumulators; lane 0 writes them, with the
// counts as 64-bit values, to row `row` of r.
template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void wave_to_lds(Acc<NP>& a, uint64_t cn, uint64_t csat, uint64_t cnf, RedLds& r,
                                            uint32_t row) {
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
    if ((threadIdx.x & 63u) == 0) {
#pragma unroll
        for (int i = 0; i < 4 * NP; ++i) r.d[row][i] = d[i];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            r.i1[row][p] = INTS ? a.i1[p] : 0;
            r.lo[row][p] = INTS ? a.i2lo[p] : 0;
            r.hi[row][p] = INTS ? a.i2hi[p] : 0;
        }
        r.c[row][0] = n;
        r.c[row][1] = sat;
        r.c[row][2] = nf;
    }
}

// Rows 0 .. nrows-1 of r added in index order (from zero) into s (all payoffs'
// fields; zero where the variant has none).
__device__ __forceinline__ void rows_total(const RedLds& r, uint32_t nrows, int np, SlotDev& s) {
    for (int p = 0; p < NPAY; ++p) {
        s.s1[p] = s.s2[p] = s.e1[p] = s.e2[p] = 0.0;
        s.i1[p] = 0;
        s.i2lo[p] = s.i2hi[p] = 0;
    }
    s.n = s.sat = s.nonfinite = s.pad = 0;
    for (uint32_t w = 0; w < nrows; ++w) {
        for (int p = 0; p < np; ++p) {
            s.s1[p] += r.d[w][p];
            s.s2[p] += r.d[w][np + p];
            s.e1[p] += r.d[w][2 * np + p];
            s.e2[p] += r.d[w][3 * np + p];
            s.i1[p] += r.i1[w][p];
            const uint64_t nlo = s.i2lo[p] + r.lo[w][p];
            s.i2hi[p] += r.hi[w][p] + (nlo < s.i2lo[p] ? 1u : 0u);
            s.i2lo[p] = nlo;
        }
        s.n += r.c[w][0];
        s.sat += r.c[w][1];
        s.nonfinite += r.c[w][2];
    }
}

// A tile's partial sums: the block sum of the per-thread accumulators (butterfly in
// each wave, then the waves in index order) written by thread 0 to *out (the
// fields the variant has).
template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void block_store(Acc<NP>& a, TileSlot* out, RedLds& r) {
    __syncthreads();                           // previous readers of r are done
    wave_to_lds<NP, CORR, INTS>(a, a.n, a.sat, a.nonfinite, r, threadIdx.x >> 6);
    __syncthreads();
    if (threadIdx.x == 0) {
        SlotDev s;
        rows_total(r, (blockDim.x + 63) >> 6, NP, s);
        out->n = s.n;
        out->sat = s.sat;
        out->nonfinite = s.nonfinite;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            PaySums& o = out->p[p];
            o.s1 = s.s1[p];
            o.s2 = s.s2[p];
            if (CORR) {
                o.e1 = s.e1[p];
                o.e2 = s.e2[p];
            }
            if (INTS) {
                o.i1 = s.i1[p];
                o.i2lo = s.i2lo[p];
                o.i2hi = s.i2hi[p];
            }
        }
    }
}

// Sums of one work item's tile slots in a fixed order that depends only on the
// number of slots: lane v of wave w (8 waves) adds slots 64 c + v for chunks
// c = w, w + 8, w + 16, ... in order; a butterfly adds each wave's lanes and the
// waves are added in index order.  Only the payoffs, correction sums and integer
// sums of the work's kernel variant are added; the rest of the result is zero.
// A lane reads the counts and each payoff's sums of its slot as whole 16-byte words
// of one line.
constexpr int REDUCE_THREADS = 512;
constexpr int REDUCE_WAVES = REDUCE_THREADS / 64;

// The fields of one tile slot that a reduction adds.
template <int NP, bool CORR, bool INTS>
struct SlotPart {
    ulonglong2 c;                  // n, sat
    uint64_t nf;
    double2 s[NP], e[NP];          // (s1, s2), (e1, e2)
    ulonglong2 w[NP];              // (i2lo, i2hi)
    int64_t i1[NP];
};

template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void load_part(const TileSlot& x, SlotPart<NP, CORR, INTS>& v) {
    v.c = *reinterpret_cast<const ulonglong2*>(&x.n);
    v.nf = x.nonfinite;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        v.s[p] = *reinterpret_cast<const double2*>(&x.p[p].s1);
        if (CORR) v.e[p] = *reinterpret_cast<const double2*>(&x.p[p].e1);
        if (INTS) {
            v.w[p] = *reinterpret_cast<const ulonglong2*>(&x.p[p].i2lo);
            v.i1[p] = x.p[p].i1;
        }
    }
}

// Slots in flight per lane of a reduction: a lane loads its next red_batch slots
// (those below ns) before adding them in order, so that a work with thousands of
// tiles is not bound by one load's latency per slot (one-payoff sums: 8 slots;
// all five payoffs: 1, within the registers).
template <int NP>
constexpr uint32_t red_batch() {
    return NP == 1 ? 8u : 1u;
}

template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void reduce_work(const TileSlot* __restrict__ sl, uint32_t ns,
                                            SlotDev* __restrict__ dst, RedLds& r) {
    Acc<NP> a;
    acc_zero(a);
    uint64_t n = 0, sat = 0, nf = 0;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    constexpr uint32_t RED_BATCH = red_batch<NP>();
    for (uint32_t i0 = wave * 64u + lane; i0 < ns; i0 += RED_BATCH * REDUCE_THREADS) {
        SlotPart<NP, CORR, INTS> v[RED_BATCH];
#pragma unroll
        for (uint32_t b = 0; b < RED_BATCH; ++b)
            if (i0 + b * REDUCE_THREADS < ns) load_part(sl[i0 + b * REDUCE_THREADS], v[b]);
#pragma unroll
        for (uint32_t b = 0; b < RED_BATCH; ++b) {
            if (i0 + b * REDUCE_THREADS >= ns) break;
            n += v[b].c.x;
            sat += v[b].c.y;
            nf += v[b].nf;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                a.s1[p] += v[b].s[p].x;
                a.s2[p] += v[b].s[p].y;
                if (CORR) {
                    a.e1[p] += v[b].e[p].x;
                    a.e2[p] += v[b].e[p].y;
                }
                if (INTS) {
                    a.i1[p] += v[b].i1[p];
                    const uint64_t lo = a.i2lo[p] + v[b].w[p].x;
                    a.i2hi[p] += v[b].w[p].y + (lo < a.i2lo[p] ? 1u : 0u);
                    a.i2lo[p] = lo;
                }
            }
        }
    }
    __syncthreads();                           // previous readers of r are done
    wave_to_lds<NP, CORR, INTS>(a, n, sat, nf, r, wave);
    __syncthreads();
    if (threadIdx.x == 0) {
        SlotDev s;
        rows_total(r, REDUCE_WAVES, NP, s);
        *dst = s;
    }
}

}  // namespace mlmc
