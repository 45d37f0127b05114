// Path kernels and the level-sum reduction (Sections 2.1-2.2 of the nested MLMC
// method; per-thread work in device/paths.hpp).
//
// k_paths: blocks stride over a tile list (tile t, t + gridDim.x, ...).  For each
// tile the block loads the level's step table into LDS (when it changes), each
// thread runs path groups group_begin + tid, + blockDim, ... accumulating FP64 (and
// exact integer) sums per payoff in registers, and the block reduces them in a
// fixed order -- butterfly within each 64-lane wave, then waves in index order --
// into the tile's own slot.  k_reduce then adds each work item's slots in a fixed
// order into its result.  Results therefore do not depend on which block ran a
// tile or on what else was in the launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "device/paths.hpp"
#include "device/reduce.hpp"
#include "kernels.hpp"

namespace mlmc {

// Exact-normal kernels carry the FP64 inverse normal's constants, fixed-point kernels
// the wide integer sums and all-payoff kernels five payoffs' sums and path
// functionals: they get a 256-thread bound (more registers per lane, no spills);
// single-payoff float table-only kernels 1024.
template <int EST, int ARITH, int NP>
constexpr int max_threads() {
    return EST == MLMC_EST_APPROX && ARITH != MLMC_ARITH_FIXED && NP == 1 ? 1024 : 256;
}

template <int EST, int ARITH, bool MIL, int NP, bool TRACK, int F, bool X32>
__global__ void __attribute__((amdgpu_flat_work_group_size(64, max_threads<EST, ARITH, NP>())))
k_paths(const WorkTilesDev* __restrict__ wtiles, const uint32_t* __restrict__ counts,
        const WorkDev* __restrict__ works, const LevelDev* __restrict__ levels,
        const uint8_t* __restrict__ tables, TileSlot* __restrict__ slots) {
    const uint32_t n_wt = counts[0], n_tiles = counts[1];
    wtiles += counts[2];
    using Body = PathBody<EST, ARITH, MIL, NP, TRACK, F, X32>;
    constexpr bool CORR = EST == MLMC_EST_CORR;
    constexpr bool INTS = ARITH == MLMC_ARITH_FIXED && EST == MLMC_EST_APPROX;
    extern __shared__ __align__(16) uint8_t s_tab[];
    __shared__ RedLds red;
    __shared__ uint32_t s_ybad;
    uint32_t cur = 0xFFFFFFFFu;
    bool ytab = false;              // level-0 samples of the current level are in LDS
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDev td = tile_of(wtiles, n_wt, t);
        const WorkDev W = works[td.work];
        const LevelDev& L = levels[W.lvl];
        if (Body::HAS_TABLE && W.lvl != cur) {
            __syncthreads();
            const uint4* src = reinterpret_cast<const uint4*>(tables + L.table_off);
            uint4* dst = reinterpret_cast<uint4*>(s_tab);
            for (uint32_t i = threadIdx.x; i < (L.table_bytes >> 4); i += blockDim.x) dst[i] = src[i];
            if (threadIdx.x == 0) s_ybad = 0u;
            __syncthreads();
            cur = W.lvl;
            ytab = false;
            if (Body::YTAB && L.level == 0 && uint32_t(NP) * L.table_entries <= YTAB_MAX_ENTRIES) {
                // per-index samples of this level (after the step table)
                double* yt = reinterpret_cast<double*>(s_tab + L.table_bytes);
                for (uint32_t k = threadIdx.x; k < L.table_entries; k += blockDim.x)
                    if (!Body::ysample(L, s_tab, k, yt)) s_ybad = 1u;
                __syncthreads();
                ytab = s_ybad == 0u;
            }
        }
        Acc<NP> acc;
        acc_zero(acc);
        const uint64_t gend = td.group_begin + td.n_groups;
        if (Body::YTAB && ytab && L.level == 0) {
            const double* yt = reinterpret_cast<const double*>(s_tab + L.table_bytes);
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::ytab_group(L, W, g, s_tab, yt, acc);
        } else if (Body::HIST && L.level == 0) {
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
        } else if (Body::PAIR && L.level >= 1 && !W.debug) {
            // a thread's groups g, g + B, g + 2B, ... two at a time (packed FP16), in
            // the same order
            uint64_t g = td.group_begin + threadIdx.x;
            for (; g + blockDim.x < gend; g += 2u * blockDim.x)
                Body::run_group_pair(L, W, g, g + blockDim.x, s_tab, acc);
            if (g < gend) Body::run_group_fast(L, W, g, s_tab, acc);
        } else if ((Body::FASTG || Body::EXG) && L.level >= 1 && !W.debug) {
            // whole groups above level 0: path boundaries by construction
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::run_group_fast(L, W, g, s_tab, acc);
        } else {
            for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
                Body::run_group(L, W, g, s_tab, acc);
        }
        block_store<NP, CORR, INTS>(acc, &slots[td.slot], red);
    }
}

// Level 0 of the exact-normal estimators (plain; correction with a float table
// side) in a kernel of its own, so that its registers are allocated for this loop
// alone: a level-0 path is one step, four paths per Philox block
// (PathBody::exact0_group, the four inverse normals interleaved).  The correction
// estimator's approximate-side sample is a function of the table index, tabulated
// per level in LDS (ya_sample) after the step table.  Same per-path operations,
// tiles and block reduction as k_paths, so the sums are the same bit for bit.  At
// most five waves per SIMD for one payoff, four for all five (whose state would
// otherwise spill to scratch).
template <int EST, int ARITH, bool MIL, int NP, bool TRACK, bool X32>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NP == 1 ? 5 : 4)))
k_exact0(const WorkTilesDev* __restrict__ wtiles, const uint32_t* __restrict__ counts,
         const WorkDev* __restrict__ works, const LevelDev* __restrict__ levels,
         const uint8_t* __restrict__ tables, TileSlot* __restrict__ slots) {
    const uint32_t n_wt = counts[0], n_tiles = counts[1];
    wtiles += counts[2];
    using Body = PathBody<EST, ARITH, MIL, NP, TRACK, 1, X32>;
    static_assert(Body::EX0, "level-0 kernel of an exact-normal estimator");
    constexpr bool CORR = EST == MLMC_EST_CORR;
    extern __shared__ __align__(16) uint8_t s_tab[];
    __shared__ RedLds red;
    uint32_t cur = 0xFFFFFFFFu;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDev td = tile_of(wtiles, n_wt, t);
        const WorkDev W = works[td.work];
        const LevelDev& L = levels[W.lvl];
        if (Body::HAS_TABLE && W.lvl != cur) {
            __syncthreads();
            const uint4* src = reinterpret_cast<const uint4*>(tables + L.table_off);
            uint4* dst = reinterpret_cast<uint4*>(s_tab);
            for (uint32_t i = threadIdx.x; i < (L.table_bytes >> 4); i += blockDim.x) dst[i] = src[i];
            __syncthreads();
            double* yt = reinterpret_cast<double*>(s_tab + L.table_bytes);
            for (uint32_t k = threadIdx.x; k < L.table_entries; k += blockDim.x) Body::ya_sample(L, s_tab, k, yt);
            __syncthreads();
            cur = W.lvl;
        }
        Acc<NP> acc;
        acc_zero(acc);
        const double* yt = reinterpret_cast<const double*>(s_tab + L.table_bytes);
        const uint64_t gend = td.group_begin + td.n_groups;
        for (uint64_t g = td.group_begin + threadIdx.x; g < gend; g += blockDim.x)
            Body::exact0_group(L, W, g, s_tab, yt, acc);
        block_store<NP, CORR, false>(acc, &slots[td.slot], red);
    }
}

// Exact normals ahead of the path kernel for works with few, long paths (level >= 2,
// so a Philox block is four steps of one path): tiles are ranges of x = m P + c over
// the work's blocks in column order (c the path offset, m the block within the path,
// block b = (path_begin + c) 2^level / 4 + m).  Each thread computes one block's four
// words and their exact normals (norminv_*_x4: four chains that interleave) and
// stores them step-major (index n P + c, n = 4 m + w): consecutive
// threads take consecutive paths, so each store is a contiguous row segment and the
// path kernel reads coalesced.
template <bool F32>
__global__ void __launch_bounds__(256)
k_normals(const TileDev* __restrict__ tiles, uint32_t n_tiles, const WorkDev* __restrict__ works,
          const LevelDev* __restrict__ levels, const uint8_t* __restrict__ tables) {
    using ZT = typename std::conditional<F32, float, double>::type;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileDev td = tiles[t];
        const WorkDev W = works[td.work];
        const LevelDev& L = levels[W.lvl];
        const int lev = L.level;
        // Method 2 couples the exact side to pi(top q bits) (the correction estimator)
        const uint16_t* pi = L.perm_off ? reinterpret_cast<const uint16_t*>(tables + L.table_off + L.perm_off)
                                        : nullptr;
        const int sh = 32 - L.q;
        const uint64_t P = W.path_end - W.path_begin;
        MLMC_GLOBAL ZT* Zb = global_ptr<ZT>(W.zbuf);
        MLMC_GLOBAL uint32_t* Jb = global_ptr<uint32_t>(W.jbuf);
        const uint64_t xend = td.group_begin + td.n_groups;
        const uint64_t bpp = (uint64_t(1) << lev) / 4;              // blocks per path
        for (uint64_t x = td.group_begin + threadIdx.x; x < xend; x += blockDim.x) {
            const uint64_t m = x / P, c = x - m * P;
            const uint64_t b = (W.path_begin + c) * bpp + m;
            const u32x4 r = philox4x32_10(
                u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32), W.c2, W.c3}, W.k0, W.k1);
            const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
            uint32_t Je[4];
#pragma unroll
            for (int w = 0; w < 4; ++w)
                Je[w] = pi ? (uint32_t(pi[wd[w] >> sh]) << sh) | (wd[w] & ((1u << sh) - 1u)) : wd[w];
            ZT Z[4];
            if constexpr (F32) norminv_f32_x4(Je, Z);
            else norminv_f64_x4(Je, Z);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const uint64_t idx = (4 * m + w) * P + c;
                Jb[idx] = wd[w];
                Zb[idx] = Z[w];
            }
        }
    }
}

__global__ void __launch_bounds__(REDUCE_THREADS)
k_reduce(const TileSlot* __restrict__ slots, const ReduceDev* __restrict__ rds, SlotDev* __restrict__ results) {
    __shared__ RedLds red;
    const ReduceDev rd = rds[blockIdx.x];
    const TileSlot* sl = slots + rd.slot_begin;
    const uint32_t ns = rd.slot_end - rd.slot_begin;
    SlotDev* dst = results + rd.work;
    switch (rd.kind) {
        case 0: reduce_work<1, false, false>(sl, ns, dst, red); break;
        case 1: reduce_work<1, true, false>(sl, ns, dst, red); break;
        case 2: reduce_work<1, false, true>(sl, ns, dst, red); break;
        case 4: reduce_work<NPAY, false, false>(sl, ns, dst, red); break;
        case 5: reduce_work<NPAY, true, false>(sl, ns, dst, red); break;
        case 6: reduce_work<NPAY, false, true>(sl, ns, dst, red); break;
        default: break;
    }
}

// A flight's plan from the pinned staging buffer (coherent host memory, mapped into
// the device's address space) to device memory.  A kernel on the flight's own stream
// rather than a copy-engine transfer, so the launches behind it are ordered by that
// stream alone; system-scope loads never see a stale cached line of a reused buffer.
__global__ void __launch_bounds__(UPLOAD_THREADS)
k_upload(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, uint32_t n) {
    const uint32_t i = blockIdx.x * UPLOAD_THREADS + threadIdx.x;
    if (i < n) dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------ dispatch
using PathKernel = void (*)(const WorkTilesDev*, const uint32_t*, const WorkDev*, const LevelDev*,
                            const uint8_t*, TileSlot*);

namespace {
struct InfoOf {
    bool l0 = false;
    VariantInfo out{nullptr, 0, 0, 0};
    template <class Tag>
    void operator()(Tag) {
        using B = PathBody<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track, Tag::fields, Tag::x32>;
        if (!l0) {
            out = VariantInfo{reinterpret_cast<void*>(&k_paths<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track,
                                                               Tag::fields, Tag::x32>),
                              B::WPB, B::TAB_BYTES, max_threads<Tag::est, Tag::arith, Tag::np>()};
            return;
        }
        if constexpr (B::EX0) {
            out = VariantInfo{reinterpret_cast<void*>(
                                  &k_exact0<Tag::est, Tag::arith, Tag::mil, Tag::np, Tag::track, Tag::x32>),
                              B::WPB, B::TAB_BYTES, 256};
        }
    }
};
}  // namespace

VariantInfo variant_info(const Variant& v) {
    InfoOf f;
    f.l0 = v.l0;
    if (!dispatch_variant(v, f)) return VariantInfo{nullptr, 0, 0, 0};
    return f.out;
}

bool has_level0_kernel(const Variant& v) {
    Variant w = v;
    w.l0 = true;
    return variant_info(w).fn != nullptr;
}

hipError_t launch_paths(const VariantInfo& vi, uint32_t grid, uint32_t block, size_t lds_bytes,
                        hipStream_t st, const WorkTilesDev* wtiles, const uint32_t* counts,
                        const WorkDev* works, const LevelDev* levels, const uint8_t* tables,
                        TileSlot* slots) {
    const PathKernel k = reinterpret_cast<PathKernel>(vi.fn);
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds_bytes, st, wtiles, counts, works, levels,
                       tables, slots);
    return hipGetLastError();
}

hipError_t launch_normals(bool f32, uint32_t grid, hipStream_t st, const TileDev* tiles,
                          uint32_t n_tiles, const WorkDev* works, const LevelDev* levels,
                          const uint8_t* tables) {
    if (n_tiles == 0) return hipSuccess;
    if (f32) hipLaunchKernelGGL(k_normals<true>, dim3(grid), dim3(256), 0, st, tiles, n_tiles, works, levels, tables);
    else hipLaunchKernelGGL(k_normals<false>, dim3(grid), dim3(256), 0, st, tiles, n_tiles, works, levels, tables);
    return hipGetLastError();
}


hipError_t launch_upload(const void* host_src, void* dst, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 8 != 0 || bytes / 8 > 0xffffffffull) return hipErrorInvalidValue;
    const uint32_t n = static_cast<uint32_t>(bytes / 8);
    hipLaunchKernelGGL(k_upload, dim3((n + UPLOAD_THREADS - 1) / UPLOAD_THREADS), dim3(UPLOAD_THREADS), 0, st,
                       static_cast<const uint64_t*>(host_src), static_cast<uint64_t*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_reduce(uint32_t n, hipStream_t st, const TileSlot* slots, const ReduceDev* rds,
                         SlotDev* results) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n), dim3(REDUCE_THREADS), 0, st, slots, rds, results);
    return hipGetLastError();
}

}  // namespace mlmc
