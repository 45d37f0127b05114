// Data shared by the host runtime and the kernels (internal; not part of the ABI).
//
// A launch processes a list of tiles.  A tile is a contiguous range of "path
// groups" of one work item; a work item is one (option, level, estimator) path
// range [path_begin, path_end); a level entry holds everything the path code needs
// for one (option parameters, level, precision).  A path group is the set of paths
// whose uniforms come from whole Philox blocks: with WPB normals per block and
// N = 2^level steps per path, a group holds max(1, WPB / N) paths and
// max(N, WPB) consecutive stream positions.
#pragma once
#include <cstdint>

#include "device/fixed.hpp"
#include "../../include/mlmc.h"

namespace mlmc {

constexpr int NPAY = MLMC_NPAYOFF;

// Largest per-index sample table (payoff slots x table entries, floats) kept in LDS
// for level 0 of the FP32 approximate estimator; beyond it the index histogram.
constexpr uint32_t YTAB_MAX_ENTRIES = 4096;

// Device buffers whose addresses travel inside structs are global memory; naming
// the address space lets the compiler use global (not flat) loads and stores, which
// do not count against the LDS wait counter, so an LDS access does not have to wait
// for outstanding global loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define MLMC_GLOBAL __attribute__((address_space(1)))
#else
#define MLMC_GLOBAL
#endif
template <typename T>
__host__ __device__ __forceinline__ MLMC_GLOBAL T* global_ptr(uint64_t addr) {
    return reinterpret_cast<MLMC_GLOBAL T*>(addr);
}

// Stream positions of one path group: lcm(2^level, wpb), so that a group holds
// whole paths and whole Philox blocks (wpb = 4 * indices per word).
__host__ __device__ __forceinline__ uint64_t group_span(int level, uint32_t wpb) {
    // lcm(2^level, wpb) = wpb 2^(level - min(level, ctz(wpb)))
    if (wpb == 0) return 0;
    const int t = __builtin_ctz(wpb);
    return uint64_t(wpb) << (level - (t < level ? t : level));
}

// a / b, in 32 bits when both fit (the same quotient, cheaper on the GPU)
__host__ __device__ __forceinline__ uint64_t udiv_fast(uint64_t a, uint64_t b) {
    return ((a | b) >> 32) == 0 ? uint64_t(uint32_t(a) / uint32_t(b)) : a / b;
}

// The tiles of one work: groups [g0, g1) (S stream positions each) in nt tiles of
// `per` groups.  Groups per tile: about tile_steps path-steps, but small enough that
// the work alone has min_tiles tiles (parallelism), and at most max_tiles tiles; a
// function of the work and the geometry alone, so a work's sums do not depend on
// its neighbours (the host planner and the device sweep engine share it).
struct WorkSplit {
    uint64_t g0, g1, per, nt;
};

__host__ __device__ inline WorkSplit split_groups(uint32_t tile_steps, uint32_t min_tiles, uint32_t block,
                                                  uint64_t S, int level, uint64_t path_begin, uint64_t n,
                                                  uint64_t max_tiles) {
    WorkSplit sp;
    const uint64_t G = S >> level;                             // paths per group
    sp.g0 = udiv_fast(path_begin, G);
    sp.g1 = udiv_fast(path_begin + n - 1, G) + 1;
    const uint64_t total = sp.g1 - sp.g0;
    uint64_t ppt = udiv_fast(tile_steps, uint64_t(block) * S);
    if (ppt < 1) ppt = 1;
    const uint64_t fill = udiv_fast(total + uint64_t(block) * min_tiles - 1, uint64_t(block) * min_tiles);
    if (fill < ppt) ppt = fill;
    if (ppt < 1) ppt = 1;
    sp.per = uint64_t(block) * ppt;
    if (udiv_fast(total + sp.per - 1, sp.per) > max_tiles) sp.per = udiv_fast(total + max_tiles - 1, max_tiles);
    sp.nt = udiv_fast(total + sp.per - 1, sp.per);
    return sp;
}

struct LevelDev {
    // exact side (FP64 constants of the level)
    double con1, con1c, con2, con3, k, b;
    // FP32 side (constants rounded to FP32; f2con3 = 2 con3 for the coarse cross term)
    float fcon1, fcon1c, fcon2, fcon3, fk, fb, f2con3, fpad;
    // FP16 side (constants rounded once from FP64 to binary16)
    _Float16 hcon1, hcon1c, hcon2, hcon3, hk, hb, hpad0, hpad1;
    // fixed-point side
    int64_t icon1, icon1c, icon2, icon3, ik, ib;
    int64_t izm_c2;           // the constant 2 in zsq's format
    int32_t fX, wX;
    FxOp op_mul2, op_addX, op_mul1, op_sum1, op_zsq, op_zm1, op_mul3, op_sum2;
    // structure
    int32_t level, scheme;
    uint32_t payoff_mask;
    int32_t payoff_single;    // payoff id of a one-payoff launch
    int32_t q;
    uint32_t table_entries;   // 2^q
    uint32_t table_off;       // byte offset of the step table in the table arena
    uint32_t table_bytes;
    uint32_t perm_off;        // byte offset of Method 2's pi (uint16 per index) in the
                              // level's table entry, 0 = none (exact side uses J)
    uint32_t pad_perm;
};

struct WorkDev {
    uint32_t lvl;             // index of its LevelDev
    uint32_t c2, c3;          // counter words: level | estimator << 8, option
    uint32_t k0, k1;          // key = seed
    uint32_t pad0;
    uint64_t path_begin, path_end;
    uint64_t debug;           // device address of mlmc_path_record[path_end - path_begin] or 0
    // Normals computed ahead by k_normals (0: computed in the path kernel): for
    // path i and step n, word J and exact normal Z at index n P + (i - path_begin),
    // P = path_end - path_begin; Z has the exact side's type.
    uint64_t zbuf, jbuf;
};

struct TileDev {
    uint32_t work;
    uint32_t slot;
    uint64_t group_begin;
    uint32_t n_groups;
    uint32_t pad;
};

// The tiles of one work in a path-kernel launch, generated on the device: tile j of
// the work covers groups [g0 + j per, min(g0 + (j + 1) per, g1)) and writes slot
// slot_begin + j; the launch numbers tiles consecutively, this work's ending at
// tile_end (exclusive).
struct WorkTilesDev {
    uint64_t g0, g1, per;
    uint32_t work;
    uint32_t tile_end;
    uint32_t slot_begin;
    uint32_t pad;
};

// Tile t of a launch from its works' descriptors (binary search on tile_end).
__host__ __device__ __forceinline__ TileDev tile_of(const WorkTilesDev* wt, uint32_t n_wt, uint32_t t) {
    uint32_t lo = 0, hi = n_wt - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (wt[mid].tile_end > t) hi = mid;
        else lo = mid + 1;
    }
    const WorkTilesDev w = wt[lo];
    const uint32_t begin = lo ? wt[lo - 1].tile_end : 0u;
    const uint64_t j = t - begin;
    TileDev td;
    td.work = w.work;
    td.slot = w.slot_begin + static_cast<uint32_t>(j);
    td.group_begin = w.g0 + j * w.per;
    const uint64_t rest = w.g1 - td.group_begin;
    td.n_groups = static_cast<uint32_t>(rest < w.per ? rest : w.per);
    td.pad = 0;
    return td;
}

// Partial or accumulated sums of one work item (all payoffs).
struct SlotDev {
    double s1[NPAY], s2[NPAY], e1[NPAY], e2[NPAY];
    int64_t i1[NPAY];
    uint64_t i2lo[NPAY], i2hi[NPAY];
    uint64_t n, sat, nonfinite, pad;
};

// A tile's partial sums: the counts, then each payoff's sums together, on 128-byte
// boundaries, so that a one-payoff tile's partial is one 128-byte line (written by
// the path kernel, read by the reduction).
struct PaySums {
    double s1, s2, e1, e2;
    uint64_t i2lo, i2hi;
    int64_t i1;
    uint64_t pad;
};
struct alignas(128) TileSlot {
    uint64_t n, sat, nonfinite, pad;
    PaySums p[NPAY];
};
static_assert(sizeof(TileSlot) == 384, "tile slot: three 128-byte lines");

struct ReduceDev {
    uint32_t slot_begin, slot_end;   // this work item's tile slots
    uint32_t kind;                   // sums present: 1 correction, 2 integer, 4 all payoffs
    uint32_t work;                   // its index: the result goes to results[work]
};

}  // namespace mlmc
