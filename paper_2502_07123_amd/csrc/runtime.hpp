// Runtime internals: the context, launch planning and execution.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlmc.h"
#include "common.hpp"
#include "host/prepare.hpp"
#include "kernels.hpp"

namespace mlmc {

// Launch geometry (chosen per device by the tuner; fixed within a context so that
// sums are reproducible).
struct Tuning {
    uint32_t block_table = 256;     // threads per block, table-only kernels
    uint32_t block_exact = 256;     // threads per block, kernels with exact normals
    uint32_t tile_steps = 1u << 16; // path-steps per tile (target)
    uint32_t blocks_per_cu = 8;     // persistent grid = CUs * blocks_per_cu (cap)
    uint32_t min_tiles = 2048;      // a work is split into at least this many tiles when it can be
    // exact-normal works with at most zb_max_paths paths (and zb_max_positions
    // stream positions) get their normals computed ahead, off the paths' chains
    uint64_t zb_max_paths = 1u << 15;
    uint64_t zb_max_positions = 1u << 22;
};

// One (option, level, estimator) path range of a launch.
struct WorkSpec {
    const mlmc_problem* prob;
    int32_t level;
    const mlmc_precision* prec;
    int32_t est;
    uint64_t seed;
    uint32_t option;
    uint64_t path_begin, n;
    uint32_t sums;                  // index in the persistent sums region
    uint64_t debug;                 // device address of records or 0
    bool accumulate;                // add onto the sums (false: overwrite them)
};

struct Server;

}  // namespace mlmc

struct mlmc_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_ws = false;
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    std::string err;
    bool poisoned = false;
    uint8_t* pinned = nullptr;
    size_t pinned_bytes = 0;
    int cu_count = 0;
    mlmc::Tuning tune;
    std::mutex dev_mtx;             // one launch sequence at a time on the device
    std::unique_ptr<mlmc::Server> server;
    // per-context cache of prepared levels (key: problem, level, precision, estimator)
    std::map<std::string, mlmc::LevelPrep> prep_cache;
    // kernel timing (HIP events around each path-kernel launch)
    bool timing = false;
    std::vector<hipEvent_t> events;
    std::vector<mlmc_kernel_stat> stats;
    mlmc_context();                 // both defined where Server is complete
    ~mlmc_context();
};

namespace mlmc {

mlmc_status fail(mlmc_context* ctx, mlmc_status s, const std::string& msg);

// Runs the works as one launch sequence: path kernels (one per variant), the
// reduction into sums[0 .. n_sums) of the workspace (added onto the previous
// contents for works with accumulate), and a copy of each work's updated sums to
// out (host, one SlotDev per work, in order).
mlmc_status run_works(mlmc_context* ctx, const std::vector<WorkSpec>& works, uint32_t n_sums,
                      std::vector<SlotDev>& out);
mlmc_status estimate_batch(mlmc_context* ctx, uint32_t n, const mlmc_problem* probs,
                           const mlmc_run_config* cfg, uint64_t seed, const uint32_t* ids,
                           mlmc_result* out);

void slot_to_sums(const SlotDev& s, int np_slot, mlmc_sums& o);
mlmc_status validate_run(const mlmc_problem* prob, const mlmc_run_config* cfg, std::string& err);

// Adaptive nested MLMC for a set of options advancing in lockstep sweeps.
struct OptionRun {
    mlmc_problem prob;
    mlmc_run_config cfg;
    uint64_t seed = 0;
    uint32_t option = 0;
    uint32_t sums_base = 0;         // first of (L_max + 1) * 3 sums
    int L = 0;
    bool done = false;
    int sweeps = 0;
    double t_start = 0.0, t_end = 0.0;
    uint64_t path_steps = 0;
    uint64_t saturations = 0;
    std::vector<std::array<SlotDev, 3>> sums;   // host copy per level, estimator
};

void option_init(OptionRun& o);
// Pending (level, estimator, extra samples) of an option, or none when done.
struct Pending {
    int level, est;
    uint64_t n;
};
std::vector<Pending> option_advance(OptionRun& o);
void option_result(const OptionRun& o, mlmc_result& r);
mlmc_status run_sweeps(mlmc_context* ctx, std::vector<OptionRun*>& opts, uint32_t n_sums);
double now_seconds();

}  // namespace mlmc
