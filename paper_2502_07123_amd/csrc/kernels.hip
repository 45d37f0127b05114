// Path kernels and the level-sum reduction (Sections 2.1-2.2 of the nested MLMC
// method; per-thread work in device/paths.hpp).
//
// k_paths: blocks stride over a tile list (tile t, t + gridDim.x, ...).  For each
// tile the block loads the level's step table into LDS (when it changes), each
// thread runs path groups group_begin + tid, + blockDim, ... accumulating FP64 (and
// exact integer) sums per payoff in registers, and the block reduces them in a
// fixed order -- butterfly within each 64-lane wave, then waves in index order --
// into the tile's own slot.  Results therefore do not depend on which block ran a
// tile or on what else was in the launch.
// k_reduce: one block per work item; thread f adds field f of the item's tile
// slots sequentially in tile order (optionally onto the running total).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "device/paths.hpp"
#include "kernels.hpp"

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

template <int NP, bool CORR, bool INTS>
__device__ __forceinline__ void block_store(Acc<NP>& a, SlotDev* out, RedLds& r) {
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
    const int64_t n = wave_sum(static_cast<int64_t>(a.n));
    const int64_t sat = wave_sum(static_cast<int64_t>(a.sat));
    const int64_t nf = wave_sum(static_cast<int64_t>(a.nonfinite));
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
        *out = s;
    }
}

// Exact-normal kernels carry the FP64 inverse normal's constants: they get a
// 256-thread bound (more registers per lane, no spills); table-only kernels 1024.
template <int EST, int ARITH>
constexpr int max_threads() { return EST == MLMC_EST_APPROX ? 1024 : 256; }

template <int EST, int ARITH, bool MIL, int NP, bool TRACK, int F>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, max_threads<EST, ARITH>())))
k_paths(const TileDev* __restrict__ tiles, uint32_t n_tiles, const WorkDev* __restrict__ works,
        const LevelDev* __restrict__ levels, const uint8_t* __restrict__ tables,
        SlotDev* __restrict__ slots) {
    using Body = PathBody<EST, ARITH, MIL, NP, TRACK, F>;
    extern __shared__ __align__(16) uint8_t s_tab[];
    __shared__ RedLds red;
    uint32_t cur = 0xFFFFFFFFu;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDev td = tiles[t];
        const WorkDev W = works[td.work];
        const LevelDev& L = levels[W.lvl];
        if (Body::HAS_TABLE && W.lvl != cur) {
            __syncthreads();
            const uint4* src = reinterpret_cast<const uint4*>(tables + L.table_off);
            uint4* dst = reinterpret_cast<uint4*>(s_tab);
            for (uint32_t i = threadIdx.x; i < (L.table_bytes >> 4); i += blockDim.x) dst[i] = src[i];
            __syncthreads();
            cur = W.lvl;
        }
        Acc<NP> acc;
        acc_zero(acc);
        const uint64_t gend = td.group_begin + td.n_groups;
        for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
            Body::run_group(L, W, g, s_tab, acc);
        block_store<NP, EST == MLMC_EST_CORR, ARITH == MLMC_ARITH_FIXED && EST == MLMC_EST_APPROX>(
            acc, &slots[td.slot], red);
    }
}

__global__ void __launch_bounds__(64)
k_reduce(const SlotDev* __restrict__ slots, const ReduceDev* __restrict__ rds, uint32_t n,
         SlotDev* __restrict__ sums, SlotDev* __restrict__ compact) {
    const uint32_t w = blockIdx.x;
    if (w >= n) return;
    const ReduceDev rd = rds[w];
    SlotDev* dst = &sums[rd.sums];
    const int f = threadIdx.x;
    if (f < 4 * NPAY) {
        const int which = f / NPAY, p = f % NPAY;
        double* d = (which == 0 ? dst->s1 : which == 1 ? dst->s2 : which == 2 ? dst->e1 : dst->e2) + p;
        const size_t off = reinterpret_cast<const uint8_t*>(d) - reinterpret_cast<const uint8_t*>(dst);
        double acc = rd.accumulate ? *d : 0.0;
        for (uint32_t s = rd.slot_begin; s < rd.slot_end; ++s)
            acc += *reinterpret_cast<const double*>(reinterpret_cast<const uint8_t*>(&slots[s]) + off);
        *d = acc;
    } else if (f < 5 * NPAY) {
        const int p = f - 4 * NPAY;
        int64_t acc = rd.accumulate ? dst->i1[p] : 0;
        for (uint32_t s = rd.slot_begin; s < rd.slot_end; ++s) acc += slots[s].i1[p];
        dst->i1[p] = acc;
    } else if (f < 6 * NPAY) {
        const int p = f - 5 * NPAY;
        uint64_t lo = rd.accumulate ? dst->i2lo[p] : 0, hi = rd.accumulate ? dst->i2hi[p] : 0;
        for (uint32_t s = rd.slot_begin; s < rd.slot_end; ++s) {
            const uint64_t nlo = lo + slots[s].i2lo[p];
            hi += slots[s].i2hi[p] + (nlo < lo ? 1u : 0u);
            lo = nlo;
        }
        dst->i2lo[p] = lo;
        dst->i2hi[p] = hi;
    } else if (f < 6 * NPAY + 3) {
        const int c = f - 6 * NPAY;
        uint64_t acc = rd.accumulate ? (c == 0 ? dst->n : c == 1 ? dst->sat : dst->nonfinite) : 0;
        for (uint32_t s = rd.slot_begin; s < rd.slot_end; ++s)
            acc += c == 0 ? slots[s].n : c == 1 ? slots[s].sat : slots[s].nonfinite;
        if (c == 0) dst->n = acc;
        else if (c == 1) dst->sat = acc;
        else dst->nonfinite = acc;
    }
    __syncthreads();
    // copy the updated sums for the host (one 8-byte word per thread)
    const uint64_t* src = reinterpret_cast<const uint64_t*>(dst);
    uint64_t* cp = reinterpret_cast<uint64_t*>(&compact[w]);
    for (uint32_t i = threadIdx.x; i < sizeof(SlotDev) / 8; i += blockDim.x) cp[i] = src[i];
}

// ------------------------------------------------------------------ dispatch
using PathKernel = void (*)(const TileDev*, uint32_t, const WorkDev*, const LevelDev*,
                            const uint8_t*, SlotDev*);

namespace {
struct InfoOf {
    VariantInfo out{nullptr, 0, 0, 0};
    template <class Tag>
    void operator()(Tag) {
        using B = PathBody<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track, Tag::fields>;
        out = VariantInfo{reinterpret_cast<void*>(
                              &k_paths<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track, Tag::fields>),
                          B::WPB, B::TAB_BYTES, max_threads<Tag::est, Tag::arith>()};
    }
};
}  // namespace

VariantInfo variant_info(const Variant& v) {
    InfoOf f;
    if (!dispatch_variant(v, f)) return VariantInfo{nullptr, 0, 0, 0};
    return f.out;
}

hipError_t launch_paths(const VariantInfo& vi, uint32_t grid, uint32_t block, size_t lds_bytes,
                        hipStream_t st, const TileDev* tiles, uint32_t n_tiles,
                        const WorkDev* works, const LevelDev* levels, const uint8_t* tables,
                        SlotDev* slots) {
    const PathKernel k = reinterpret_cast<PathKernel>(vi.fn);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, st, tiles, n_tiles, works, levels,
                       tables, slots);
    return hipGetLastError();
}

hipError_t launch_reduce(uint32_t n, hipStream_t st, const SlotDev* slots, const ReduceDev* rds,
                         SlotDev* sums, SlotDev* compact) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n), dim3(64), 0, st, slots, rds, n, sums, compact);
    return hipGetLastError();
}

}  // namespace mlmc
