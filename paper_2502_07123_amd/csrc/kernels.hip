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
// k_reduce: one block per work item adds the item's tile slots in a fixed order
// (optionally onto the running total).
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
        if (Body::HIST && L.level == 0) {
            // level-0 approximate samples: count table indices in LDS, then add
            // c_k copies of each index's sample (thread t takes k = t, t + B, ...)
            uint32_t* hist = reinterpret_cast<uint32_t*>(s_tab + L.table_bytes);
            for (uint32_t i = threadIdx.x; i < L.table_entries; i += blockDim.x) hist[i] = 0u;
            __syncthreads();
            auto count = [&](uint32_t k) { atomicAdd(&hist[k], 1u); };
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::hist_group(L, W, g, s_tab, count);
            __syncthreads();
            for (uint32_t k = threadIdx.x; k < L.table_entries; k += blockDim.x) {
                const uint32_t c = hist[k];
                if (c) Body::hist_accumulate(L, s_tab, k, c, acc);
            }
        } else if (Body::HAS_EXACT && W.zbuf) {
            // normals computed ahead: a group is one path
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::run_path_buffered(L, W, g, s_tab, acc);
        } else {
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::run_group(L, W, g, s_tab, acc);
        }
        block_store<NP, EST == MLMC_EST_CORR, ARITH == MLMC_ARITH_FIXED && EST == MLMC_EST_APPROX>(
            acc, &slots[td.slot], red);
    }
}

// Exact normals ahead of the path kernel for works with few, long paths: tiles
// are ranges of Philox blocks b of the work's stream (positions 4b .. 4b + 3);
// each thread computes one block's four words and their exact normals and stores
// them step-major (index n P + path offset) so the path kernel reads coalesced.
template <bool F32>
__global__ void __launch_bounds__(256)
k_normals(const TileDev* __restrict__ tiles, uint32_t n_tiles, const WorkDev* __restrict__ works,
          const LevelDev* __restrict__ levels) {
    using ZT = typename std::conditional<F32, float, double>::type;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDev td = tiles[t];
        const WorkDev W = works[td.work];
        const int lev = levels[W.lvl].level;
        const uint64_t P = W.path_end - W.path_begin;
        ZT* Zb = reinterpret_cast<ZT*>(W.zbuf);
        uint32_t* Jb = reinterpret_cast<uint32_t*>(W.jbuf);
        const uint64_t bend = td.group_begin + td.n_groups;
        for (uint64_t b = td.group_begin + threadIdx.x; b < bend; b += blockDim.x) {
            const u32x4 r = philox4x32_10(
                u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), W.c2, W.c3}, W.k0, W.k1);
            const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll 1
            for (int w = 0; w < 4; ++w) {
                const uint64_t g = 4 * b + w;
                const uint64_t i = g >> lev, n = g & ((uint64_t(1) << lev) - 1);
                const uint64_t idx = n * P + (i - W.path_begin);
                Jb[idx] = wd[w];
                if (F32) Zb[idx] = static_cast<ZT>(norminv_f32(wd[w]));
                else Zb[idx] = static_cast<ZT>(norminv_f64(wd[w]));
            }
        }
    }
}

// Sums of one work's tile slots in a fixed order: thread t adds slots t, t + B,
// t + 2B, ... (B = 256), then a butterfly within each wave and the waves in index
// order, onto the running total when accumulating.
struct RedAcc {
    double d[4 * NPAY];
    int64_t i1[NPAY];
    uint64_t lo[NPAY], hi[NPAY];
    uint64_t c[3];
};

__device__ __forceinline__ void red_zero(RedAcc& a) {
#pragma unroll
    for (int i = 0; i < 4 * NPAY; ++i) a.d[i] = 0.0;
#pragma unroll
    for (int p = 0; p < NPAY; ++p) { a.i1[p] = 0; a.lo[p] = 0; a.hi[p] = 0; }
    a.c[0] = a.c[1] = a.c[2] = 0;
}

__device__ __forceinline__ void add128(uint64_t& lo, uint64_t& hi, uint64_t blo, uint64_t bhi) {
    const uint64_t nlo = lo + blo;
    hi += bhi + (nlo < lo ? 1u : 0u);
    lo = nlo;
}

__device__ __forceinline__ void red_add(RedAcc& a, const SlotDev& s) {
#pragma unroll
    for (int p = 0; p < NPAY; ++p) {
        a.d[p] += s.s1[p];
        a.d[NPAY + p] += s.s2[p];
        a.d[2 * NPAY + p] += s.e1[p];
        a.d[3 * NPAY + p] += s.e2[p];
        a.i1[p] += s.i1[p];
        add128(a.lo[p], a.hi[p], s.i2lo[p], s.i2hi[p]);
    }
    a.c[0] += s.n;
    a.c[1] += s.sat;
    a.c[2] += s.nonfinite;
}

__device__ __forceinline__ void red_add(RedAcc& a, const RedAcc& b) {
#pragma unroll
    for (int i = 0; i < 4 * NPAY; ++i) a.d[i] += b.d[i];
#pragma unroll
    for (int p = 0; p < NPAY; ++p) { a.i1[p] += b.i1[p]; add128(a.lo[p], a.hi[p], b.lo[p], b.hi[p]); }
    a.c[0] += b.c[0];
    a.c[1] += b.c[1];
    a.c[2] += b.c[2];
}

__device__ __forceinline__ void red_wave(RedAcc& a) {
#pragma unroll
    for (int i = 0; i < 4 * NPAY; ++i) a.d[i] = wave_sum(a.d[i]);
#pragma unroll
    for (int p = 0; p < NPAY; ++p) {
        a.i1[p] = wave_sum(a.i1[p]);
        wave_sum128(a.lo[p], a.hi[p]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) a.c[i] = static_cast<uint64_t>(wave_sum(static_cast<int64_t>(a.c[i])));
}

constexpr int REDUCE_THREADS = 256;

__global__ void __launch_bounds__(REDUCE_THREADS)
k_reduce(const SlotDev* __restrict__ slots, const ReduceDev* __restrict__ rds, uint32_t n,
         SlotDev* __restrict__ sums, SlotDev* __restrict__ compact) {
    __shared__ RedAcc part[REDUCE_THREADS / 64];
    const uint32_t w = blockIdx.x;
    if (w >= n) return;
    const ReduceDev rd = rds[w];
    SlotDev* dst = &sums[rd.sums];
    RedAcc a;
    red_zero(a);
    for (uint32_t s = rd.slot_begin + threadIdx.x; s < rd.slot_end; s += blockDim.x) red_add(a, slots[s]);
    red_wave(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        RedAcc t;
        red_zero(t);
        if (rd.accumulate) red_add(t, *dst);
        for (int v = 0; v < static_cast<int>(blockDim.x >> 6); ++v) red_add(t, part[v]);
        SlotDev o;
        for (int p = 0; p < NPAY; ++p) {
            o.s1[p] = t.d[p];
            o.s2[p] = t.d[NPAY + p];
            o.e1[p] = t.d[2 * NPAY + p];
            o.e2[p] = t.d[3 * NPAY + p];
            o.i1[p] = t.i1[p];
            o.i2lo[p] = t.lo[p];
            o.i2hi[p] = t.hi[p];
        }
        o.n = t.c[0];
        o.sat = t.c[1];
        o.nonfinite = t.c[2];
        o.pad = 0;
        *dst = o;
        compact[w] = o;
    }
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

hipError_t launch_normals(bool f32, uint32_t grid, hipStream_t st, const TileDev* tiles,
                          uint32_t n_tiles, const WorkDev* works, const LevelDev* levels) {
    if (n_tiles == 0) return hipSuccess;
    if (f32) hipLaunchKernelGGL(k_normals<true>, dim3(grid), dim3(256), 0, st, tiles, n_tiles, works, levels);
    else hipLaunchKernelGGL(k_normals<false>, dim3(grid), dim3(256), 0, st, tiles, n_tiles, works, levels);
    return hipGetLastError();
}

hipError_t launch_reduce(uint32_t n, hipStream_t st, const SlotDev* slots, const ReduceDev* rds,
                         SlotDev* sums, SlotDev* compact) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n), dim3(REDUCE_THREADS), 0, st, slots, rds, n, sums, compact);
    return hipGetLastError();
}

}  // namespace mlmc
