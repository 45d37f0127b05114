// Host side of the device sweep engine (engine.hpp), internal.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "engine.hpp"
#include "runtime.hpp"

namespace mlmc {

// a (scheme, path functionals, nested) combination the engine serves
struct EngKind {
    int scheme = 0;
    bool track = false;
    bool nested = false;
    bool operator==(const EngKind& o) const { return scheme == o.scheme && track == o.track && nested == o.nested; }
    bool operator<(const EngKind& o) const {
        return scheme != o.scheme ? scheme < o.scheme : (track != o.track ? track < o.track : nested < o.nested);
    }
};

struct EngClass {
    Variant v;
    VariantInfo vi{nullptr, 0, 0, 0};
    uint32_t block = 0, lds = 0;
};

mlmc_status engine_classes(mlmc_context* ctx, const mlmc_run_config& cfg, const std::vector<EngKind>& kinds,
                           std::vector<EngClass>& out, size_t& tstride);

struct Engine {
    mlmc_context* ctx = nullptr;
    mlmc_run_config cfg{};          // the runs' levels' precisions, plain arithmetic, L_max
    std::vector<EngKind> kinds;
    uint32_t C = 0, LV = 0;
    std::vector<EngClass> cls;
    size_t tstride = 256;           // bytes per (slot, level, table side) step table
    uint64_t slot_cap = 0;          // tile slots
    uint64_t tune_key = 0;
    EngPtrs P{};
    LevelDev* levels = nullptr;     // [slot][level][estimator]
    uint8_t* tables = nullptr;      // [slot][level][approximate, correction] * tstride
    hipStream_t st = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    uint32_t* status_h[2] = {nullptr, nullptr};   // pinned: each graph's status copy
    hipEvent_t ev_done[2] = {nullptr, nullptr};
    RunState* states_h = nullptr;                 // pinned: states downloaded at the end
    std::vector<uint32_t> levels_ready, generation;
    std::vector<EngMeta> meta_h;                  // host mirror of the host-owned meta words

    struct StageBuf {
        uint8_t* p = nullptr;
        size_t bytes = 0;
        hipEvent_t ev = nullptr;
    };
    std::vector<StageBuf> stage;                  // pinned host staging buffers
    uint8_t* dstage = nullptr;                    // device staging area (workspace)
    size_t dstage_bytes = 0;
    // base tables (Z~ values per (arith, q, method) of the runs' FP32 / FP16 table
    // sides) for the step tables built on the device, and their job list
    std::vector<uint8_t> base_h;
    std::vector<std::pair<std::tuple<int, int, int>, uint32_t>> base_index;   // key -> byte offset
    uint8_t* base = nullptr;
    EngTableJob* jobs = nullptr;
    uint32_t jobs_cap = 0;
    // An upload: segments copied by scatter launches, concurrently -- no two
    // segments of one upload may overlap.
    struct Upload {
        std::vector<uint8_t> data;
        std::vector<EngSeg> segs;
        std::vector<EngTableJob> jobs;            // step tables the device builds after the copies
        uint8_t* put(const void* src, size_t bytes, uint64_t dst);
        void zero(size_t bytes, uint64_t dst);    // bytes: multiple of 8
    };
    // levels [from, to) of the run in slot s
    struct LevelTask {
        uint32_t s;
        const mlmc_problem* prob;
        bool nested;
        uint32_t from, to;
    };

    ~Engine();
    static size_t slot_bytes(uint32_t LV, size_t tstride);
    mlmc_status build_bases();
    bool base_of(int arith, int q, int method, uint32_t& off) const;
    mlmc_status create(mlmc_context* c, const mlmc_run_config& rc, const std::vector<EngKind>& k, uint32_t n);
    mlmc_status layout();
    mlmc_status capture(int k);
    mlmc_status flush(Upload& u);
    void stage_reset(Upload& u);
    // the levels of every task, prepared on up to 8 host threads, then staged in order
    mlmc_status stage_tasks(Upload& u, const std::vector<LevelTask>& tasks);
    // With `defer`, the run's (or its more) levels are appended there for one
    // stage_tasks call over many runs; without, staged at once.
    mlmc_status stage_run(Upload& u, uint32_t s, const mlmc_problem& prob, const mlmc_run_config& rc,
                          uint64_t seed, uint32_t option, bool put_meta, std::vector<LevelTask>* defer = nullptr);
    void stage_meta_all(Upload& u);
    mlmc_status stage_more_levels(Upload& u, uint32_t s, const mlmc_problem& prob, bool nested, uint32_t need,
                                  std::vector<LevelTask>* defer = nullptr);
    void stage_levels_ready(Upload& u, uint32_t s, uint32_t c3);
    mlmc_status replay(int k);
};

// Runs the adaptive estimates of `runs` (one payoff each, the same run config's
// precisions) to completion on the device sweep engine; their states hold the sums.
mlmc_status engine_run_batch(mlmc_context* ctx, std::vector<OptionRun>& runs);

}  // namespace mlmc
