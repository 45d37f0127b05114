// Kernel variants and launch entry points (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace mlmc {

// One compiled instance of the path body: estimator, arithmetic of the table
// (or plain) side, scheme, payoffs per launch (1 or NPAY), whether Asian sums and
// running minima are kept, and indices per 32-bit word (1 = unpacked).
struct Variant {
    int est, arith, scheme, np;
    bool track;
    int fields;
    bool l0 = false;    // level-0 works of an exact-normal estimator in their own kernel
    bool exact32 = false;   // correction estimator with an FP32 exact side
};

template <int EST, int ARITH, bool MIL, int NP, bool TRACK, int F, bool X32 = false>
struct VTag {
    static constexpr int est = EST, arith = ARITH, np = NP, fields = F;
    static constexpr bool mil = MIL, track = TRACK, x32 = X32;
};

namespace detail {
template <int EST, int ARITH, bool MIL, int F, bool X32, class Fn>
bool pick_np(const Variant& v, Fn& fn) {
    if (v.np != 1) { fn(VTag<EST, ARITH, MIL, NPAY, true, F, X32>{}); return true; }
    if (v.track) { fn(VTag<EST, ARITH, MIL, 1, true, F, X32>{}); return true; }
    fn(VTag<EST, ARITH, MIL, 1, false, F, X32>{});
    return true;
}
template <int EST, int ARITH, int F, class Fn, bool X32 = false>
bool pick_mil(const Variant& v, Fn& fn) {
    return v.scheme == MLMC_MILSTEIN ? pick_np<EST, ARITH, true, F, X32>(v, fn)
                                     : pick_np<EST, ARITH, false, F, X32>(v, fn);
}
}  // namespace detail

// Calls fn(VTag<...>{}) for the compiled instance matching v; false if none.
template <class Fn>
bool dispatch_variant(const Variant& v, Fn& fn) {
    using namespace detail;
    switch (v.est) {
        case MLMC_EST_PLAIN:
            if (v.fields != 1) return false;
            if (v.arith == MLMC_ARITH_FP64) return pick_mil<MLMC_EST_PLAIN, MLMC_ARITH_FP64, 1>(v, fn);
            if (v.arith == MLMC_ARITH_FP32) return pick_mil<MLMC_EST_PLAIN, MLMC_ARITH_FP32, 1>(v, fn);
            return false;
        case MLMC_EST_APPROX:
            if (v.arith == MLMC_ARITH_FIXED)
                return v.fields == 1 && pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FIXED, 1>(v, fn);
            if (v.arith == MLMC_ARITH_FP16) {
                if (v.fields == 1) return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP16, 1>(v, fn);
                if (v.fields == 4) return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP16, 4>(v, fn);
                return false;
            }
            if (v.arith != MLMC_ARITH_FP32) return false;
            switch (v.fields) {
                case 1: return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP32, 1>(v, fn);
                case 4: return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP32, 4>(v, fn);
                case 5: return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP32, 5>(v, fn);
                case 8: return pick_mil<MLMC_EST_APPROX, MLMC_ARITH_FP32, 8>(v, fn);
                default: return false;
            }
        case MLMC_EST_CORR:
            if (v.fields != 1) return false;
            if (v.exact32) {
                // FP32 exact side (float table sides only)
                if (v.arith == MLMC_ARITH_FP32) return pick_mil<MLMC_EST_CORR, MLMC_ARITH_FP32, 1, Fn, true>(v, fn);
                if (v.arith == MLMC_ARITH_FP16) return pick_mil<MLMC_EST_CORR, MLMC_ARITH_FP16, 1, Fn, true>(v, fn);
                return false;
            }
            if (v.arith == MLMC_ARITH_FIXED) return pick_mil<MLMC_EST_CORR, MLMC_ARITH_FIXED, 1>(v, fn);
            if (v.arith == MLMC_ARITH_FP32) return pick_mil<MLMC_EST_CORR, MLMC_ARITH_FP32, 1>(v, fn);
            if (v.arith == MLMC_ARITH_FP16) return pick_mil<MLMC_EST_CORR, MLMC_ARITH_FP16, 1>(v, fn);
            return false;
        default:
            return false;
    }
}

struct VariantInfo {
    void* fn;              // kernel
    int wpb;               // normals per Philox block
    int tab_bytes;         // bytes per table entry (0: no table)
    int max_block;         // largest block size the kernel was compiled for
};

VariantInfo variant_info(const Variant& v);   // fn == nullptr when not compiled

// Whether level-0 works of variant v (no debug records, level 0, table of at most
// YTAB_MAX_ENTRIES payoff slots x entries) run in the level-0 kernel.
bool has_level0_kernel(const Variant& v);

// counts[1] tiles generated from counts[0] work descriptors starting at
// wtiles + counts[2] (tile_of); counts is device memory, read by the kernel (a
// captured launch reads its sizes at run time)
hipError_t launch_paths(const VariantInfo& vi, uint32_t grid, uint32_t block, size_t lds_bytes,
                        hipStream_t st, const WorkTilesDev* wtiles, const uint32_t* counts,
                        const WorkDev* works, const LevelDev* levels, const uint8_t* tables,
                        TileSlot* slots);

// Philox blocks per tile of the normals-ahead kernel (one per thread of its 256)
constexpr uint64_t NORMALS_TILE_BLOCKS = 256;

// exact normals ahead of the path kernel (FP32 for the plain-FP32 estimator, else FP64)
hipError_t launch_normals(bool f32, uint32_t grid, hipStream_t st, const TileDev* tiles,
                          uint32_t n_tiles, const WorkDev* works, const LevelDev* levels,
                          const uint8_t* tables);

// copies `bytes` (a multiple of 8) from coherent pinned host memory to device memory
// with a kernel on `st`
constexpr uint32_t UPLOAD_THREADS = 256;
hipError_t launch_upload(const void* host_src, void* dst, size_t bytes, hipStream_t st);

// results[rds[b].work] = fixed-order sum of that work's tile slots (block b of n
// takes rds[b]); results may be device memory or coherent pinned host memory (the
// sums then reach the host with the kernel's completion, without a copy)
hipError_t launch_reduce(uint32_t n, hipStream_t st, const TileSlot* slots, const ReduceDev* rds,
                         SlotDev* results);

}  // namespace mlmc
