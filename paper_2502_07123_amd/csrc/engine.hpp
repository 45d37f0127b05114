// The device sweep engine: the adaptive MLMC runs of many options kept on the GPU.
//
// Each run (an option being priced to its eps) owns a slot: its RunState (sums per
// (level, estimator), sample counts -- the next path index of each uniform stream
// -- and the driver's decisions), its prepared levels (constants and step tables)
// and their launch classes.  One sweep is a fixed sequence of kernels, captured once
// in a HIP graph and replayed:
//   k_eng_advance  one block per slot: the driver's next works (device/advance.hpp:
//                  pilot, per-level estimator, optimal allocation, bias test);
//   k_eng_plan     one block: the works of all slots into per-class work lists and
//                  tile descriptors (the same tile split as a host-planned launch),
//                  path offsets from the runs' sample counts;
//   k_paths / k_exact0 per class (persistent; sizes read from device memory);
//   k_eng_reduce   each work's tile sums in the fixed order, added into its run's
//                  sums (the sample counts advance with them);
//   a copy of the slots' status words to host memory.
// The host replays the graph, prepares levels a run reaches (a run waits for a level
// that is not prepared yet) and collects finished runs.  The decisions and sums are
// those of the host-driven driver bit for bit: the same run_advance code on the same
// sums, the same tiles and the same fixed-order reductions.
#pragma once
#include <cstdint>

#include "common.hpp"
#include "device/advance.hpp"

namespace mlmc {

constexpr int ENG_MAX_CLASSES = 24;

// status word of a slot (EngMeta::status)
constexpr uint32_t ENG_DONE = 1u;          // the run has finished
constexpr uint32_t ENG_WAIT_LEVEL = 2u;    // its next works need a level not prepared yet

struct EngHeader {
    uint32_t n_slots;           // C
    uint32_t n_levels;          // levels per slot (L_max + 1)
    uint32_t n_classes;
    uint32_t tile_steps, min_tiles;
    uint32_t max_tiles_work;    // tiles per work at most
    uint32_t n_works;           // this sweep's works (k_eng_plan)
    uint32_t error;             // 1: one run's works need more tile slots than the engine has
    uint64_t slot_cap;          // tile slots
    uint64_t max_works;         // C * RUN_MAX_PEND
    uint32_t planned, deferred; // this sweep: runs planned, runs deferred (capacity)
    uint32_t pad0, pad1;
    uint32_t counts[ENG_MAX_CLASSES][4];      // per class: work descriptors, tiles, first descriptor, 0
    uint32_t class_work_off[ENG_MAX_CLASSES]; // first work / first tile slot of each class
    uint32_t class_slot_off[ENG_MAX_CLASSES];
};

struct EngMeta {
    uint32_t active;            // host: the slot holds a run
    uint32_t pending_valid;     // device: pend[] holds works not run yet
    uint32_t levels_ready;      // host: levels 0 .. levels_ready - 1 are prepared
    uint32_t c3;                // option id (uniform counter word)
    uint32_t k0, k1;            // seed (key)
    uint32_t status;            // device: ENG_* bits; bits 8..15 the level waited for
    uint32_t generation;        // host: bumped when the slot gets a new run
};

// launch class and split parameters of one (slot, level, estimator)
struct EngLevelInfo {
    uint16_t cls;
    uint16_t wpb;
    uint16_t block;
    uint16_t kind;              // reduction: 1 correction sums, 2 exact integer sums
};

struct EngReduce {
    uint32_t slot_begin, slot_end;
    uint32_t kind;
    uint32_t run;
    int32_t level, est;
    uint64_t n;
};

// one pending work of a run as the sweep plans it (written by k_eng_advance, read by
// k_eng_plan)
struct EngWorkPlan {
    WorkSplit sp;                 // its tile split
    uint64_t begin, n;            // path range [begin, begin + n) of its stream
    int32_t level, est;
    uint32_t cls, kind;           // launch class, reduction kind
    uint32_t iw, t0;              // its place in its class's list and its first tile there
};

// per-slot planning scratch
struct EngPlanScratch {
    uint64_t total_tiles;         // the run's pending works' tiles
    uint32_t planned;
    int32_t need;                 // highest level of a pending work not prepared yet (-1: none)
    uint32_t bad;                 // a pending work's level has no launch class
    uint32_t n_works;
    EngWorkPlan w[RUN_MAX_PEND];
};

// device addresses of an engine's arrays (kernel arguments)
struct EngPtrs {
    EngHeader* hdr;
    RunState* states;
    EngMeta* meta;
    EngLevelInfo* info;         // [slot][level][estimator]
    EngPlanScratch* scratch;    // [slot]
    WorkDev* works;             // [max_works]
    WorkTilesDev* wtiles;       // [max_works], each class's in one run (counts[c][2] on)
    EngReduce* red;             // [max_works]
    TileSlot* slots;            // [slot_cap]
    uint32_t* status_out;       // [slot] status words for the host, then the error word
};

// one contiguous piece of a host-to-device upload (engine_kernels k_scatter)
struct EngSeg {
    uint64_t src;               // byte offset in the staging area (multiple of 8), or ENG_SEG_ZERO
    uint64_t dst;               // device address (multiple of 8)
    uint64_t bytes;             // multiple of 8
};
constexpr uint64_t ENG_SEG_ZERO = ~uint64_t(0);   // the segment's bytes are zeros

// A step table built on the device: the (Z~_k, s_k) pairs of one (slot, level)'s
// FP32 or FP16 table side, Z~_k from the engine's base table of the precision's
// (q, method) and s_k the fine step's multiplier with that level's constants -- the
// same operations as the host's table build (device/paths.hpp multiplier_lp).
struct EngTableJob {
    uint32_t lvl;               // LevelDev index [slot][level][estimator]
    uint32_t table_off;         // destination, bytes into the table arena
    uint32_t base_off;          // Z~ values, bytes into the base table area
    uint16_t arith;             // MLMC_ARITH_FP32 or MLMC_ARITH_FP16
    uint16_t mil;               // Milstein multiplier
};

hipError_t launch_eng_tables(const EngTableJob* jobs, uint32_t n, const LevelDev* levels, const uint8_t* base,
                             uint8_t* tables, hipStream_t st);
hipError_t launch_eng_advance(const EngPtrs& p, uint32_t n_slots, hipStream_t st);
hipError_t launch_eng_plan(const EngPtrs& p, hipStream_t st);
hipError_t launch_eng_reduce(const EngPtrs& p, uint32_t grid, hipStream_t st);
// copies n segments from a device staging area (staging + segs, device memory) to
// their destinations
hipError_t launch_eng_scatter(const uint8_t* staging, const EngSeg* segs, uint32_t n, hipStream_t st);

}  // namespace mlmc
